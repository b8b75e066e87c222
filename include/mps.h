/*
 * mps.h -- C ABI of libmps, a gfx950 (MI355X) implementation of multiway
 * Powersort (Cawley Gelling, Nebel, Smith, Wild, "Multiway Powersort",
 * arXiv 2209.06909).
 *
 * What the library computes is the paper's problem statement (Section 1 and
 * Section 2): stably sort an array by first finding its existing runs
 * (maximal weakly increasing or strictly decreasing segments; decreasing
 * runs are reversed), giving every run boundary its k-way node power
 * (Definition 3.1), and merging the runs k-way along the merge tree those
 * powers define (Algorithm 1; Algorithm 2 builds the same tree).  The result
 * is the unique stable sort: equal keys keep their input order.
 *
 * Conventions shared by every entry point:
 *  - Pointers named keys / payload / offsets are DEVICE pointers (memory of
 *    the current HIP device); trace buffers are HOST pointers.
 *  - The caller owns keys, payload and offsets; they are sorted in place and
 *    must stay valid until the work enqueued on `stream` has finished.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls only enqueue work unless a trace is requested (then they wait).
 *  - Keys are int32, int64 or float32.  float32 keys are ordered by the
 *    IEEE-754 total order (-0 before +0, NaNs by bit pattern).  The payload
 *    is an optional uint32 per key that moves with its key (NULL: keys only).
 *  - Errors found on the host are returned as negative mps_status codes
 *    before any work is enqueued; mps_last_error() gives a message for the
 *    calling thread.  The kernels also check the consistency of what they
 *    build (run table, merge tree, co-ranks, tile descriptors) and record a
 *    failed check in the sort's device-side error word, whose output must
 *    then not be trusted.  That word reaches the caller in three ways: a
 *    trace request (the call returns MPS_E_DEVICE), mps_sort_status() after
 *    the sort (it synchronises), or mps_opts.error_out (a device word the
 *    sort ORs its error bits into, without synchronising).  HIP runtime
 *    faults surface at the caller's next synchronisation.
 *  - Workspace: every sort needs device scratch memory
 *    (mps_workspace_bytes).  Either the caller passes it in
 *    mps_opts.workspace -- one workspace must not be used by two sorts that
 *    can run at the same time, e.g. on two streams -- or the library keeps
 *    one per (device, stream), allocated on first use and kept until
 *    mps_free_workspaces().  Growing a library-managed workspace
 *    synchronises its stream and frees the old allocation, so a call that
 *    needs a larger one is not asynchronous.
 */
#ifndef MPS_H
#define MPS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MPS_OK = 0,
    MPS_PENDING = 1,          /* serving: request not finished yet */
    MPS_E_INVALID = -1,       /* bad argument (NULL pointer with n > 0, bad offsets, ...) */
    MPS_E_NOMEM = -2,         /* workspace too small / allocation failed / over budget */
    MPS_E_HIP = -3,           /* a HIP runtime call failed */
    MPS_E_UNSUPPORTED = -4,   /* k not in {2,4,8}, an array longer than 2^31, ... */
    MPS_E_NOTFOUND = -5,      /* serving: unknown request id */
    MPS_E_DEVICE = -6         /* a device-side consistency check failed */
} mps_status;

typedef enum { MPS_I32 = 0, MPS_I64 = 1, MPS_F32 = 2 } mps_key_type;

/* Option flags (mps_opts.flags). */
#define MPS_OPT_TIME_LEVELS 1u  /* record HIP events around every level's co-rank and merge
                                   launches (read them with mps_last_level_stats) */
#define MPS_OPT_GRAPH 2u        /* capture the call's launch sequence in a HIP graph the first
                                   time these exact arguments (pointers, sizes, options) are
                                   seen and replay the graph on later calls; the graph reads
                                   every data-dependent quantity on the device, so new
                                   contents of keys / payload / offsets are fine.  Not with
                                   MPS_OPT_TIME_LEVELS. */
#define MPS_OPT_MERGE_DOWN 4u   /* the final phase of the paper's 4-way implementation
                                   (Appendix A.3) instead of Algorithm 2's: with s runs left on
                                   the stack after the last one, the top s mod (k-1) are merged
                                   with it first, then k-1 at a time, so every later merge is
                                   k-way.  Only the nodes along the tree's right spine change,
                                   and the merge cost never rises.  Each such node reports the
                                   power of its first boundary, and so do its boundaries in the
                                   trace.  Single arrays only (batched: MPS_E_UNSUPPORTED); a
                                   no-op for k = 2. */
#define MPS_OPT_TEST_DEVICE_ERROR 8u /* testing only: the sort runs normally but reports a
                                   failed device-side check (bit 30 of the error word), to
                                   exercise the caller's error path */

/* Options.  All fields may be zero for defaults.  The defaults of k, tile and
 * lane_slice can be set per process from the environment: MPS_K (2, 4 or 8),
 * MPS_TILE (1024, 2048 or 4096) and MPS_LANE_SLICE (4 or 8), read once at the
 * first call; unsupported values are ignored, and a lane slice that does not
 * pair with the tile falls back to 4. */
typedef struct {
    uint32_t k;                 /* merge arity: 2, 4 (default, the paper's 4-way) or 8 */
    uint32_t flags;             /* MPS_OPT_* bits */
    void *workspace;            /* device memory of >= mps_workspace_bytes(); NULL: the
                                   library allocates and caches one per (device, stream) */
    uint64_t workspace_bytes;
    uint32_t tile;              /* merge tile, outputs per workgroup task: 1024, 2048
                                   (default) or 4096 */
    uint32_t lane_slice;        /* outputs each thread merges per LDS stage (tile divided by
                                   the workgroup size): 4 or 8; 0 = 4.  Valid pairs: 1024/4,
                                   2048/8, 2048/4, 4096/8, 4096/4 */
    uint32_t min_run;           /* minimal run length (Appendix A.3; the paper's experiments
                                   use 24).  0 or 1: natural runs.  2..32: scanning left to
                                   right, a natural run shorter than min_run is extended to
                                   min(n, start + min_run) elements, which are sorted stably
                                   (the order an insertion sort gives), and the next run
                                   starts where it ends; powers and the merge tree are those
                                   of the extended runs.  Single-array sorts only (batched:
                                   MPS_E_UNSUPPORTED); above 32: MPS_E_UNSUPPORTED. */
    uint32_t *error_out;        /* device uint32 or NULL: after the sort, a last kernel on the
                                   stream ORs the sort's device-side error bits into it (0:
                                   every check passed).  The caller clears it; it is sticky
                                   across sorts, and works with MPS_OPT_GRAPH. */
} mps_opts;

/* What the sort did (filled when a trace pointer is passed; forces a stream
 * synchronisation).  Counters are always filled; each array is filled only
 * if the caller supplies it (host memory, room for r_cap runs / nodes;
 * MPS_E_NOMEM if r_cap is too small). */
typedef struct {
    uint64_t r;                 /* runs found (Section 2) */
    uint64_t n_nodes;           /* internal merge-tree nodes */
    uint64_t merge_cost;        /* sum of all merge output sizes (Section 2.3) */
    uint32_t n_levels;          /* 1 + depth of the deepest internal node */
    uint32_t k;                 /* arity used */
    uint64_t r_cap;             /* capacity of the arrays below, in runs */
    uint64_t *run_start;        /* [r+1] first position of every run, run_start[r] = n */
    uint8_t *run_desc;          /* [r] 1 if the run was strictly decreasing */
    uint8_t *power;             /* [r-1] power[i-1] = P_i of the boundary starting run i
                                   (0 where a boundary is also an array edge in a batch) */
    uint8_t *leaf_depth;        /* [r] depth of every run in the merge tree */
    uint64_t *node_begin;       /* [n_nodes] element span of every node ... */
    uint64_t *node_end;         /*            ... in order of their leftmost boundary */
    uint32_t *node_first;       /* [n_nodes] leftmost boundary index of the node */
    uint8_t *node_arity;        /* [n_nodes] number of children (2..k) */
    uint8_t *node_power;        /* [n_nodes] common power of the node's boundaries */
    uint8_t *node_depth;        /* [n_nodes] depth (root = 0) */
} mps_trace;

/* Bytes of device workspace needed to sort n elements in m arrays with the
 * given key type, payload and arity.  has_payload: 0 none, 1 a u32 payload,
 * 2 a u64 payload (mps_sort_kv64, single arrays only).  Returns 0 on bad
 * arguments. */
uint64_t mps_workspace_bytes(uint64_t n, uint64_t m, mps_key_type kt, int has_payload,
                             uint32_t k);

/* Stable multiway Powersort of one array of n keys (and payloads) in place:
 * run detection and reversal (Section 2), node powers (Definition 3.1),
 * merge tree (Algorithm 1), k-way merges along the tree.  n <= 1 is a no-op;
 * n > 2^31 gives MPS_E_UNSUPPORTED; keys == NULL with n > 0 gives
 * MPS_E_INVALID. */
int mps_sort(void *keys, mps_key_type kt, uint32_t *payload, uint64_t n, void *stream);
int mps_sort_i32(int32_t *keys, uint32_t *payload, uint64_t n, void *stream);
int mps_sort_i64(int64_t *keys, uint32_t *payload, uint64_t n, void *stream);
int mps_sort_f32(float *keys, uint32_t *payload, uint64_t n, void *stream);

/* mps_sort with options and an optional trace (trace may be NULL). */
int mps_sort_ex(void *keys, mps_key_type kt, uint32_t *payload, uint64_t n,
                const mps_opts *opts, mps_trace *trace, void *stream);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the sort of
 * mps_sort_ex (same result, same options) with its workspace in a fixed
 * device array of the library, mps_noalloc_scratch_bytes() = 64 MiB, that
 * every device the library runs on holds from the first such call until the
 * process ends.  The call allocates nothing: no hipMalloc / hipFree, no HIP
 * events, streams or graphs, no host memory.
 *  - Limit: mps_workspace_bytes(n, 1, kt, payload != NULL, k) must not exceed
 *    the scratch (about 2.2M int64 or 1.9M int32/float32 keys with a u32
 *    payload at k = 4); larger sorts return MPS_E_NOMEM before any work is
 *    enqueued.
 *  - opts may be NULL.  opts->workspace must be NULL (MPS_E_INVALID);
 *    MPS_OPT_GRAPH and MPS_OPT_TIME_LEVELS give MPS_E_UNSUPPORTED (they create
 *    HIP objects).  There is no trace; device-side check results reach the
 *    caller through opts->error_out.
 *  - Every call on a device shares that device's scratch, which keeps the last
 *    call's contents (the sort clears what it needs cleared itself).  Calls
 *    that can overlap on one device -- on two streams, or from two threads --
 *    race on it and must be serialised by the caller.
 * Errors otherwise as mps_sort_ex. */
int mps_sort_noalloc(void *keys, mps_key_type kt, uint32_t *payload, uint64_t n,
                     const mps_opts *opts, void *stream);
uint64_t mps_noalloc_scratch_bytes(void);

/* Records of a key and an 8-byte payload, such as the key-and-pointer records
 * of the paper's experiments with 16-byte records (Section 4): the stable sort
 * of mps_sort_ex, with payload (device, n u64) permuted with the keys.  The
 * merges carry each 8-byte payload with its key (mps_workspace_bytes with
 * has_payload = 2: an 8-byte ping-pong payload buffer, 4 bytes per key more
 * than a u32 payload).  Options, trace, limits and errors as mps_sort_ex;
 * payload NULL or n <= 1 is mps_sort_ex without a payload. */
int mps_sort_kv64(void *keys, mps_key_type kt, uint64_t *payload, uint64_t n,
                  const mps_opts *opts, mps_trace *trace, void *stream);

/* Batched: m independent arrays packed back to back, array i occupying
 * [offsets[i], offsets[i+1]) of keys/payload (offsets: device uint64[m+1],
 * offsets[0] = 0, non-decreasing, offsets[m] = total_n; empty arrays are
 * allowed).  Every array is sorted on its own, exactly as mps_sort would sort
 * it alone: runs never cross an array edge and every power is normalised by
 * its own array's length (Definition 3.1).  All arrays go through one shared
 * sequence of launches, one per tree level.  h_offsets (host copy, nullable)
 * is used only to validate; each array must hold at most 2^31 keys. */
int mps_sort_batched(void *keys, mps_key_type kt, uint32_t *payload, const uint64_t *offsets,
                     const uint64_t *h_offsets, uint64_t m, uint64_t total_n,
                     const mps_opts *opts, mps_trace *trace, void *stream);

/* Autotuner for batched sorts (a systems layer; the paper has no such step).
 * Times every candidate configuration -- arity k in {4, 2, 8} times the tile
 * configurations (tile, lane_slice) in {2048/8, 1024/4, 2048/4, 4096/8,
 * 4096/4}, in that order -- on a sample of the batch (whole arrays from the start, up to
 * sample_cap keys; 0 = 2^27) and writes the fastest into best->k, best->tile
 * and best->lane_slice (other fields untouched).  keys / payload are the
 * batch's device arrays (read only; the sample is copied), h_offsets its host
 * offsets [m+1].  flags: 0 or MPS_OPT_GRAPH (time graph replays, as a caller
 * using MPS_OPT_GRAPH will run).  cand_ms (nullable, 15 floats) receives every
 * candidate's mean time in ms.  The choice is cached per device, key type,
 * payload presence, log2(total keys) and log2(mean array size); a cached
 * choice is returned without timing unless cand_ms is requested.  If the
 * environment variable MPS_AUTOTUNE_CACHE names a file, choices persist there
 * across processes (one JSON object per line: GPU architecture name, key type,
 * payload presence, both size buckets, graph flag, k, tile, lane_slice); the
 * file is read at the first call on each device and every new choice is
 * appended.  Allocates
 * tuner memory (about twice the sample plus a workspace) for the duration of
 * the call and synchronises `stream`.  Note that k changes the merge tree
 * (powers are base-k), never the sorted result. */
int mps_autotune(const void *keys, mps_key_type kt, const uint32_t *payload,
                 const uint64_t *h_offsets, uint64_t m, uint64_t sample_cap, uint32_t flags,
                 mps_opts *best, float *cand_ms, void *stream);

/* Outcome of the device-side checks of the most recent sort that used
 * `workspace` (the opts->workspace of that call; NULL: the library-managed
 * workspace of the current device and `stream`).  Synchronises `stream`
 * first.  MPS_OK if every check passed, MPS_E_DEVICE if one failed (that
 * sort's output must not be trusted; the message gives the error word),
 * MPS_E_NOTFOUND if no sort has used the library-managed workspace of this
 * device and stream.  The error word is reset by the next sort that uses
 * the same workspace. */
int mps_sort_status(const void *workspace, void *stream);

/* Synchronises every device that holds a library-managed workspace and frees
 * them all (the next sort on a stream allocates a new one).  Traces and level
 * timings of sorts that used them can no longer be fetched. */
int mps_free_workspaces(void);

/* Fills trace (counters and every array the caller supplies) from the most
 * recent sort that used `workspace` (the opts->workspace pointer of that
 * call; NULL: the library-managed workspace of the current device).  Lets a
 * caller learn r and n_nodes first and size the host arrays afterwards.
 * Synchronises the device.  MPS_E_NOTFOUND if no such sort exists. */
int mps_trace_fetch(const void *workspace, mps_trace *trace);

/* Per-level figures of the most recent sort on the current device that was
 * run with MPS_OPT_TIME_LEVELS: the number of levels run by the level merges
 * (1 + the deepest depth of a node whose span exceeds 1024 elements; the
 * smaller subtrees are finished by one pass before the levels and are not
 * counted), and for each level d < min(cap, n_levels) the number of elements
 * the level merges output
 * (the level's share of the merge cost, Section 2.3) and the durations of
 * its co-rank and merge launches in milliseconds (HIP events on the sort's
 * stream).  Any output pointer may be NULL.  Waits for that sort to finish.
 * MPS_E_NOTFOUND if there was no such sort. */
int mps_last_level_stats(uint32_t cap, uint32_t *n_levels, uint64_t *level_elems,
                         float *corank_ms, float *merge_ms);

/* A streaming device-to-device copy of `bytes` bytes from src to dst (device
 * pointers, both 16-byte aligned, not overlapping), enqueued on `stream`:
 * 16-byte loads and stores, every byte read once and written once.  Not part
 * of the sort; it is the measuring stick for the HBM bandwidth that a one-pass
 * kernel reaches on the device (the benchmark's copy ceiling, and the copy of
 * known size that calibrates the traffic counters).  MPS_E_INVALID for a NULL
 * or misaligned pointer. */
int mps_stream_copy(const void *src, void *dst, uint64_t bytes, void *stream);

/* ------------------------------------------------------------ serving
 * A continuous-batching server (a systems layer around the sort; the paper has
 * none).  Requests are device-resident and caller-owned; submit never blocks
 * on the GPU.  A scheduler thread admits queued requests in arrival order
 * into batches whose device memory -- packed copies of the requests plus the
 * batched sort's workspace -- fits in the free part of an arena of
 * hbm_budget_bytes reserved at creation.  Each batch runs on one of n_streams
 * streams (gather, one mps_sort_batched, scatter), so batches formed from
 * requests that arrived meanwhile overlap on the device.  Each result is
 * exactly what mps_sort gives for that request alone.  The server uses the
 * device that is current when it is created. */
typedef struct mps_server mps_server;

typedef struct {
    uint64_t hbm_budget_bytes;  /* device arena for admitted requests (allocated once) */
    uint32_t n_streams;         /* batches in flight at once (0: 2; at most 16) */
    uint32_t max_batch;         /* requests per batch (0: 256) */
    uint32_t k;                 /* merge arity (0: 4) */
    uint32_t tile, lane_slice;  /* merge tile configuration (0: defaults, as mps_opts) */
    uint32_t poll_us;           /* scheduler wake-up period while batches run (0: 20 us) */
    uint32_t fail_every;        /* testing: every fail_every-th batch is failed on the host
                                   before anything is enqueued (0: never) */
} mps_serve_cfg;

typedef struct {
    const void *keys;           /* device, n keys (read only) */
    const uint32_t *payload;    /* device, n payloads, or NULL */
    void *keys_out;             /* device, n keys: the sorted keys (may equal keys) */
    uint32_t *payload_out;      /* device, NULL iff payload is NULL (may equal payload) */
    uint64_t n;                 /* <= 2^31 */
    mps_key_type kt;
    void *ready_event;          /* hipEvent_t or NULL: the batch's stream waits for it before
                                   reading the inputs (e.g. recorded after the work that
                                   produced them); must stay valid until completion */
} mps_request;

typedef struct {
    uint64_t t_submit_ns;       /* host steady clock at submit */
    uint64_t t_admit_ns;        /* when its batch was formed and enqueued */
    uint64_t t_done_ns;         /* when the scheduler saw the batch complete */
    uint64_t batch;             /* batch number (from 1) */
    uint32_t batch_requests;    /* requests in that batch */
    int status;                 /* MPS_PENDING, MPS_OK or an error */
} mps_req_info;

typedef struct {
    uint64_t queued;            /* submitted, not yet admitted */
    uint64_t batches;           /* batches launched so far */
    uint64_t arena_bytes, arena_used;
    uint32_t busy_streams;
} mps_serve_stats_t;

/* MPS_E_INVALID (bad cfg), MPS_E_UNSUPPORTED, MPS_E_NOMEM (budget above the
 * free device memory, or allocation failure), MPS_E_HIP. */
int mps_serve_create(const mps_serve_cfg *cfg, mps_server **out);
/* Queues a request; *req_id identifies it.  The caller keeps every buffer valid
 * until poll reports completion.  MPS_E_INVALID for NULL pointers or a payload
 * without payload_out, MPS_E_NOMEM if the request alone needs more than the
 * whole budget, MPS_E_UNSUPPORTED for n > 2^31. */
int mps_serve_submit(mps_server *s, const mps_request *req, uint64_t *req_id);
/* Status of a request (MPS_PENDING, MPS_OK, or the error that ended it --
 * MPS_E_HIP for a failed launch, MPS_E_DEVICE for a failed device-side
 * check); info (nullable) receives its timestamps.  MPS_E_NOTFOUND for an
 * unknown or released id. */
int mps_serve_poll(mps_server *s, uint64_t req_id, mps_req_info *info);
/* Forgets a finished request (MPS_E_INVALID if it is still pending). */
int mps_serve_release(mps_server *s, uint64_t req_id);
int mps_serve_stats(mps_server *s, mps_serve_stats_t *stats);
/* Stops accepting requests, finishes every queued and running one, and frees
 * the server. */
int mps_serve_destroy(mps_server *s);
/* Host-only self-test of the server's arena allocator and batching policy
 * (needs no GPU): 0, or the number of the first failed check. */
int mps_serve_selftest(void);

/* Message describing the last error of the calling thread ("" if none). */
const char *mps_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
