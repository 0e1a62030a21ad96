/*
 * leiden.h - C ABI of the MI355X (gfx950) dynamic Leiden library.
 *
 * Community detection on an evolving undirected graph with the Leiden method
 * and its three dynamic front-ends, Naive-dynamic (ND), Delta-screening (DS)
 * and Dynamic Frontier (DF), as defined in Sahu, "A Starting Point for Dynamic
 * Community Detection with Leiden Algorithm" (arXiv 2405.11658):
 *   - problem statement and update call: Sec. 3.5 and Sec. 4.5 (the update
 *     takes G^t, the batch Delta^-, Delta^+, C^{t-1}, K^{t-1}, Sigma^{t-1} and
 *     returns C^t, K^t, Sigma^t);
 *   - modularity: Eq. 1; move score: Eq. 2;
 *   - pass loop: Alg. "leiden"; phases: Alg. "leidenMove", "leidenRefine",
 *     "leidenAggregate", "leidenSubsetRenumber"; weights: Alg. "updateWeights";
 *   - front-ends: Alg. "naiveDynamic", "deltaScreening", "dynamicFrontier".
 *
 * Conventions.  Graphs are CSR: int64 offsets [n+1], int32 neighbour ids,
 * float32 weights (> 0).  An undirected graph stores both directions of every
 * edge; a self-loop (i,i,w) is stored once and counts w once.  Weight totals
 * (K, Sigma, 2m) and modularity are float64 (Sec. 5.1.2).
 *
 * Memory.  Unless a parameter says "host", every pointer is a device pointer
 * (device memory of the current device).  The caller owns all input and
 * output buffers; they must stay valid until the work enqueued on `stream`
 * completes.  A handle owns its graph, state and scratch, obtained from the
 * allocator given to leiden_create (else from HIP's stream-ordered allocator);
 * leiden_destroy releases them.  `stream` is a hipStream_t passed as void*
 * (NULL = default stream).
 *
 * Ordering.  Calls are stream-ordered; calls that return host values (q_out,
 * stats, counts) synchronise the stream before returning.  A call on a handle
 * enqueued on another stream than the handle's previous call first waits (on
 * the device) for the previous call's work.  No call waits for the whole
 * device: memory is released in stream order.
 *
 * Errors.  Every entry point returns a leiden_status; no exception crosses the
 * ABI.  On LEIDEN_EINVAL the handle is unchanged (inputs are validated before
 * any mutation).  A LEIDEN_ENOMEM or LEIDEN_EHIP from leiden_update after the
 * batch was validated leaves the handle holding G^t without a community state:
 * its next leiden_update returns LEIDEN_ESTATE until leiden_static or
 * leiden_set_state installs a membership again.  leiden_last_error() gives a
 * message for the last failure on a handle.
 *
 * Concurrency.  A handle is used by one host thread at a time; distinct
 * handles are independent.
 */
#ifndef LEIDEN_H
#define LEIDEN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LEIDEN_OK = 0,
  LEIDEN_EINVAL = 1, /* bad argument, id out of range, non-positive weight,
                        malformed batch (see leiden_batch) */
  LEIDEN_ENOMEM = 2, /* device allocation failed */
  LEIDEN_ESTATE = 3, /* update before leiden_static / leiden_set_state */
  LEIDEN_EHIP = 4    /* HIP runtime error */
} leiden_status;

/* Dynamic front-ends (Sec. 3.5.1-3.5.3, Appendix A.1-A.2, Sec. 4.5). */
typedef enum { LEIDEN_ND = 1, LEIDEN_DS = 2, LEIDEN_DF = 3 } leiden_mode;

/* Parameters (Sec. 4.6 and 5.1.2).  leiden_default_params fills the paper's
 * values: tau0 = 0.01, tol_drop = 10, max_iter = 20; max_passes = 10 (not
 * stated in the paper); agg_tol = 1.0 (aggregation never skipped, Sec. 4.6).
 * sync_mode = 0 (default): asynchronous local moving and refinement as in
 * Sec. 4.6 - up to async_waves wavefronts (0 = 4096; at most one per 1024
 * vertices with edges on the first level, per 256 on aggregated levels) sweep
 * the vertices in ascending id order and apply each move at once; results
 * depend on timing.
 * Vertices of degree > hub_degree (default 256: those whose neighbour table
 * does not fit a wavefront's LDS table) are moved before each sweep by several
 * workgroups each, synchronously within each of hub_slices hash-ordered slices
 * (0 = 64; more slices move fewer hubs at once).  sync_mode = 1: deterministic test
 * mode - every vertex is swept in nslices hash-ordered slices (default 16),
 * the slices in order, the vertices of a slice synchronously, the gain summed
 * in a fixed order; results are bit-identical to the CPU oracle's synchronous
 * mode.  refine_variant: 0 Subset Refine
 * (Sec. 4.3, default), 1 Full Refine (Sec. 4.2), 2 no continued passes
 * (Sec. 4.1).  profile = 1 times selected kernels with HIP events on the
 * call's stream (see leiden_stats.prof_*); results are unaffected. */
typedef struct {
  double tau0;
  double tol_drop;
  double agg_tol;
  int32_t max_iter;
  int32_t max_passes;
  int32_t sync_mode;
  int32_t refine_variant;
  int32_t nslices; /* 1 .. 256, synchronous mode */
  int32_t profile; /* 0 or 1 */
  int32_t async_waves; /* 0 .. 65536; 1 = one wavefront: the serial sweep */
  int32_t hub_slices;  /* 0 .. 256, asynchronous mode only */
  int32_t verts_per_wave;        /* asynchronous sweeps: vertices with edges per
                                    wavefront on the first level (0 = 1024) */
  int32_t verts_per_wave_upper;  /* the same on aggregated levels (0 = 256) */
  int32_t hub_degree;  /* asynchronous mode: vertices of higher degree move in
                          the hub slices before each sweep (default 256;
                          64 .. 2048; 0 = 2048) */
  int32_t trim;        /* 1: every call releases its working buffers when it
                          ends (stream-ordered; the graph and the community
                          state stay), for many resident graphs; 0: kept */
} leiden_params;

#define LEIDEN_MAX_PASSES 64

/* Kernels timed when leiden_params.profile = 1 (index into leiden_stats.prof_*):
 *   HUB_GATHER  - local moving of the hubs (degree > hub_degree): asynchronous
 *                 mode, every slice of an iteration (gather, score and apply
 *                 kernels) timed as one region; synchronous mode, the gather
 *                 launch of each slice with hubs; entries = edges scanned by
 *                 the gathers;
 *   AGG_MERGE   - the aggregation of a level up to its row lengths (several
 *                 kernels, timed as one region per aggregated level);
 *                 entries = level CSR entries, vertices = level vertices;
 *   MOD_SCAN    - modularity edge scan; entries / vertices of the graph;
 *   BATCH_MERGE - graph update merge of the old rows with the batch;
 *                 entries = CSR entries of G^t, vertices = n;
 *   MOVE_SWEEP  - asynchronous local-moving sweep, one launch per iteration;
 *                 entries = edges scanned, vertices = vertices evaluated;
 *   REFINE_SWEEP - asynchronous refinement sweep, one launch per pass;
 *                 entries = edges scanned, vertices = candidates evaluated. */
enum {
  LEIDEN_PROF_HUB_GATHER = 0,
  LEIDEN_PROF_AGG_MERGE = 1,
  LEIDEN_PROF_MOD_SCAN = 2,
  LEIDEN_PROF_BATCH_MERGE = 3,
  LEIDEN_PROF_MOVE_SWEEP = 4,
  LEIDEN_PROF_REFINE_SWEEP = 5,
  LEIDEN_PROF_N = 6
};

/* Per-call statistics (host struct). */
typedef struct {
  int32_t passes;
  int32_t move_iters[LEIDEN_MAX_PASSES];
  int32_t refine_rounds[LEIDEN_MAX_PASSES];
  int64_t level_vertices[LEIDEN_MAX_PASSES];
  int64_t level_entries[LEIDEN_MAX_PASSES];
  int64_t communities[LEIDEN_MAX_PASSES];
  int64_t refined_vertices[LEIDEN_MAX_PASSES];
  int64_t affected;     /* vertices initially marked affected */
  int64_t changed;      /* communities flagged changed after the first local-moving phase */
  int64_t moves_pass0;  /* moves in the first local-moving phase */
  double ms_total;      /* device time of the call (HIP events on `stream`) */
  double ms_apply;      /* batch validation + graph update (not in the paper's timing) */
  double ms_mark;       /* marking, changedCommunities, updateWeights */
  double ms_move;
  double ms_refine;
  double ms_aggregate;
  double ms_other;      /* renumber, lookup, final relabel, Sigma recompute, modularity */
  /* with leiden_params.profile = 1: per timed kernel, the number of launches,
   * their summed duration (HIP events around each launch) and the work they
   * covered; zero otherwise. */
  int64_t prof_launches[LEIDEN_PROF_N];
  double prof_ms[LEIDEN_PROF_N];
  int64_t prof_entries[LEIDEN_PROF_N];
  int64_t prof_vertices[LEIDEN_PROF_N];
  /* device time of each pass's local-moving, refinement and aggregation */
  double pass_move_ms[LEIDEN_MAX_PASSES];
  double pass_refine_ms[LEIDEN_MAX_PASSES];
  double pass_agg_ms[LEIDEN_MAX_PASSES];
} leiden_stats;

/* Batch update (Sec. 3.5, Sec. 5.1.4).  Device arrays; each undirected edge
 * is listed once, in either orientation; the library applies both
 * directions.  A deleted edge must exist in G^{t-1} (its weight is taken
 * from the graph); an inserted edge must not; no self-loops, no repeated
 * edge, ids in [0, n), inserted weights finite and > 0.  Anything else is
 * LEIDEN_EINVAL and leaves the handle unchanged. */
typedef struct {
  int64_t n_del;
  const int32_t *del_u;
  const int32_t *del_v;
  int64_t n_ins;
  const int32_t *ins_u;
  const int32_t *ins_v;
  const float *ins_w;
} leiden_batch;

/* Optional trace of an update (device arrays of n bytes, each nullable):
 * affected = deltaV after marking (isAffected), in_range = inAffectedRange,
 * changed = changed-community flags from changedCommunities (keyed by the
 * previous community id). */
typedef struct {
  uint8_t *affected;
  uint8_t *in_range;
  uint8_t *changed;
} leiden_trace;

typedef struct leiden_handle leiden_handle;

/* Device-memory provider of a handle (for example a framework's caching
 * allocator).  alloc returns `bytes` of device memory usable by work enqueued
 * on `stream` (a hipStream_t as void*), or NULL when it cannot; the library
 * then fails the call with LEIDEN_ENOMEM.  release returns memory that alloc
 * gave out (same size); it is called without waiting for the device, with
 * the stream that last used the memory, after that use was enqueued: the
 * provider must not hand the memory to other work before the work enqueued
 * on that stream so far has completed.  Both may be called from the library's
 * worker threads (leiden_update_many, leiden_server_*), never concurrently
 * for one handle. */
typedef struct {
  void *(*alloc)(void *ctx, size_t bytes, void *stream);
  void (*release)(void *ctx, void *ptr, size_t bytes, void *stream);
  void *ctx;
} leiden_allocator;

void leiden_default_params(leiden_params *p /* host */);

/* Create a handle holding a copy of the graph (rows are sorted by the
 * library; duplicate entries in a row are LEIDEN_EINVAL).  params may be NULL
 * for the defaults.  alloc (host struct, copied; may be NULL) provides every
 * device allocation of the handle for its whole life; NULL uses HIP's
 * stream-ordered allocator (hipMallocAsync / hipFreeAsync).  *out (host)
 * receives the handle. */
leiden_status leiden_create(int64_t n, int64_t nnz, const int64_t *offsets, const int32_t *indices,
                            const float *weights, const leiden_params *params, const leiden_allocator *alloc,
                            void *stream, leiden_handle **out);

/* Releases the handle's memory in stream order after its last enqueued work
 * (no wait for the device); the handle pointer is invalid afterwards. */
leiden_status leiden_destroy(leiden_handle *h);

leiden_status leiden_set_params(leiden_handle *h, const leiden_params *params /* host */);

/* Static Leiden (Alg. "leiden" from singletons, everything affected and
 * changed).  membership_out: n int32, dense labels in [0, |Gamma|) ascending
 * by final label; nullable.  q_out (host, nullable): Eq. 1 of the result.
 * stats (host, nullable).  Stores C, K, Sigma, 2m in the handle. */
leiden_status leiden_static(leiden_handle *h, int32_t *membership_out, double *q_out,
                            leiden_stats *stats, void *stream);

/* Dynamic update: apply the batch to the handle's graph (G^t), then run the
 * ND / DS / DF front-end and the pass loop from the stored membership.
 * Outputs as for leiden_static; trace nullable.  Requires a prior
 * leiden_static or leiden_set_state (else LEIDEN_ESTATE). */
leiden_status leiden_update(leiden_handle *h, const leiden_batch *batch, int32_t mode,
                            int32_t *membership_out, double *q_out, leiden_stats *stats,
                            const leiden_trace *trace, void *stream);

/* Marking only (Alg. "naiveDynamic", "deltaScreening", "dynamicFrontier",
 * and changedCommunities of Alg. "leiden"): the flags leiden_update would
 * compute for this batch - affected (deltaV), in_range (inAffectedRange) and
 * changed (keyed by the previous community id), each n bytes, nullable - from
 * G^t (the handle's graph with the batch applied), the stored C^{t-1},
 * K^{t-1}, Sigma^{t-1} and 2m.  The batch is validated as for leiden_update.
 * Pure: the handle's graph and state are not modified (its scratch is).
 * Requires a prior leiden_static or leiden_set_state (else LEIDEN_ESTATE). */
leiden_status leiden_mark_affected(leiden_handle *h, const leiden_batch *batch, int32_t mode,
                                   uint8_t *affected, uint8_t *in_range, uint8_t *changed, void *stream);

/* Estimate (host, *bytes) of the device memory a leiden_update with n_del
 * deletions and n_ins insertions may newly allocate on this handle: the
 * update's working set for the grown graph minus what the handle holds.
 * Used by the server's admission; an estimate, not a bound. */
leiden_status leiden_update_bytes(const leiden_handle *h, int64_t n_del, int64_t n_ins, int64_t *bytes /* host */);

/* Batched form of leiden_update for many independent graphs (the update of
 * Sec. 3.5 applied to each).  handles[k] (host array of distinct handles),
 * batches[k], modes[k] and, when non-NULL, membership_out[k] (host array of
 * device pointers), q_out[k] (host), stats[k] (host) and status_out[k]
 * (host) are as for one leiden_update call.  The updates run concurrently,
 * each on a library-created stream driven by one of max_parallel host worker
 * threads (0 = 8, at most 64), ordered after the work already enqueued on
 * `stream`; `stream` waits for all of them.  A failing update does not stop
 * the others; the return value is the first non-OK status in index order.
 * A handle listed twice is LEIDEN_EINVAL (nothing runs). */
leiden_status leiden_update_many(leiden_handle *const *handles, const leiden_batch *batches,
                                 const int32_t *modes, int32_t count, int32_t *const *membership_out,
                                 double *q_out, leiden_stats *stats, leiden_status *status_out,
                                 int32_t max_parallel, void *stream);

/* Serving loop over many resident graphs (handles): update requests are
 * queued by leiden_server_submit and run as they are admitted - up to
 * `slots` at a time (1 .. 64), each on a stream and host worker of its own,
 * while the summed device-memory estimate of the running requests (each the
 * leiden_update_bytes of its handle and batch, taken at admission) stays
 * within memory_budget bytes (0 = unlimited; a request is always admitted
 * when nothing else runs) and no other request of the same handle runs.  A
 * request that does not fit lets later ones that do go first.  The batch
 * arrays and membership_out (device, nullable) must stay valid, and the
 * handle must not be used by the caller, until leiden_server_wait for the
 * request returns.  wait blocks until the request is done and returns its
 * status, modularity, stats (host, each nullable), the latency from
 * submission to completion and the service time (host clock, ms); each id
 * can be waited for once.  destroy finishes every submitted request first. */
typedef struct leiden_server leiden_server;
leiden_status leiden_server_create(int32_t slots, int64_t memory_budget, leiden_server **out);
leiden_status leiden_server_submit(leiden_server *server, leiden_handle *h, const leiden_batch *batch,
                                   int32_t mode, int32_t *membership_out, int64_t *request_id /* host */);
/* A job for graph `graph` of a fleet (mode 0 static, or LEIDEN_ND / DS / DF
 * with batch; see leiden_fleet_run).  Queued fleet jobs are gathered into
 * one launch when a slot takes the first of them: every later queued job of
 * the same fleet on another graph joins it (a graph's jobs run in submission
 * order, one per launch); the fleet runs one launch at a time.  The batch and
 * membership_out (device, nullable) must stay valid, and the fleet must not
 * be used by the caller, until leiden_server_wait for the request returns;
 * the reported service time is the launch's. */
struct leiden_fleet;
leiden_status leiden_server_submit_fleet(leiden_server *server, struct leiden_fleet *fleet, int32_t graph,
                                         const leiden_batch *batch, int32_t mode, int32_t *membership_out,
                                         int64_t *request_id /* host */);
leiden_status leiden_server_wait(leiden_server *server, int64_t request_id, leiden_status *status,
                                 double *q_out, leiden_stats *stats, double *latency_ms,
                                 double *service_ms);
leiden_status leiden_server_destroy(leiden_server *server);

/* Fleet: many small graphs updated together in one persistent launch.
 *
 * A fleet holds `count` graphs (each as leiden_create copies it: CSR with
 * int64 offsets, int32 ids, float32 weights; rows need not be sorted) and
 * their community state in device memory.  leiden_fleet_run takes a list of
 * jobs - graph index graphs[k] (each at most once per run) and mode modes[k]:
 * 0 static Leiden (Alg. "leiden" from singletons), LEIDEN_ND / DS / DF an
 * update with batches[k] (as for leiden_update; a graph needs a static job or
 * an earlier update first, else that job's status is LEIDEN_ESTATE) - and
 * runs all of them in ONE launch: each workgroup takes jobs from a queue and
 * performs a whole update of one graph (graph update, marking,
 * changedCommunities, updateWeights, the pass loop, final relabel, Sigma and
 * Eq. 1).  The launch is replayed from a captured HIP graph.
 *
 * Local moving and refinement are the serial asynchronous sweeps of
 * Alg. "leidenMove" and "leidenRefine" (vertices one at a time in ascending
 * id order, the workgroup sharing each vertex's edges and table), so every
 * job's result is determined by its graph and batch alone - equal to the
 * serial reading of the paper's algorithms, and independent of the launch
 * variant (leiden_fleet_set_variant: wavefronts per workgroup and LDS table
 * slots, a speed choice only; leiden_fleet_variant_info describes it).
 * params: as for leiden_create (sync_mode, nslices, async_waves, hub_slices
 * and profile are not used; max_passes <= 16).  alloc as for leiden_create.
 *
 * Per job, when the arrays are non-NULL: membership_out[k] (device, n of
 * that graph, dense labels), q_out[k], status_out[k] and stats[k] (host;
 * passes, move_iters, level_vertices, communities, affected, changed,
 * moves_pass0, ms_total = the launch's device time).  *ms_out (host,
 * nullable): device time of the launch.  The return value is the first
 * non-OK job status (the other jobs still ran); a malformed call (graph index
 * out of range or repeated, bad mode, NULL batch arrays) is LEIDEN_EINVAL and
 * runs nothing.  An invalid batch leaves its graph unchanged.  A graph's
 * buffers grow (stream-ordered) when a batch would exceed their capacity. */
typedef struct leiden_fleet leiden_fleet;
leiden_status leiden_fleet_create(int32_t count, const int64_t *n /* host */, const int64_t *nnz /* host */,
                                  const int64_t *const *offsets, const int32_t *const *indices,
                                  const float *const *weights /* host arrays of device pointers */,
                                  const leiden_params *params, const leiden_allocator *alloc, void *stream,
                                  leiden_fleet **out);
leiden_status leiden_fleet_run(leiden_fleet *fleet, int32_t count, const int32_t *graphs /* host */,
                               const int32_t *modes /* host */, const leiden_batch *batches /* host */,
                               int32_t *const *membership_out, double *q_out, leiden_status *status_out,
                               leiden_stats *stats, double *ms_out, void *stream);
leiden_status leiden_fleet_get_graph(leiden_fleet *fleet, int32_t graph, int64_t *offsets, int32_t *indices,
                                     float *weights, int64_t *nnz /* host */, void *stream);
leiden_status leiden_fleet_get_state(leiden_fleet *fleet, int32_t graph, int32_t *membership, double *K,
                                     double *Sigma, double *m2 /* host */, void *stream);
leiden_status leiden_fleet_set_variant(leiden_fleet *fleet, int32_t variant /* 0 .. 5 */);
leiden_status leiden_fleet_variant_info(int32_t variant, int32_t *waves /* host */, int32_t *slots /* host */);
int32_t leiden_fleet_count(const leiden_fleet *fleet);
const char *leiden_fleet_last_error(const leiden_fleet *fleet);
leiden_status leiden_fleet_destroy(leiden_fleet *fleet);

/* Eq. 1 in FP64 for any CSR graph and membership (labels in [0, n));
 * q_out (host) is 0 when the graph has no edges.  Stateless. */
leiden_status leiden_modularity(int64_t n, const int64_t *offsets, const int32_t *indices,
                                const float *weights, const int32_t *membership, double *q_out,
                                void *stream);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): Eq. 1 as
 * leiden_modularity computes it, with nnz given by the caller and the result
 * written to q_out in device memory (NaN when a label or neighbour id is out
 * of [0, n)).  Nothing is allocated, freed or waited for: the working arrays
 * live in one fixed array of the library per device (64 MiB, held until the
 * process ends), which every call on that device shares and which keeps the
 * last call's contents - calls that overlap on one device race.  n above
 * leiden_modularity_noalloc_max_vertices() (8,388,576) is LEIDEN_EINVAL and
 * enqueues nothing. */
leiden_status leiden_modularity_noalloc(int64_t n, int64_t nnz, const int64_t *offsets, const int32_t *indices,
                                        const float *weights, const int32_t *membership, double *q_out /* device */,
                                        void *stream);
int64_t leiden_modularity_noalloc_max_vertices(void);

/* Alg. "leidenAggregate" for a given membership with dense labels in
 * [0, ncomm): super-vertex CSR with, for each pair of communities, the FP64
 * sum of the weights rounded to float32.  out_offsets: ncomm+1 int64;
 * out_indices / out_weights: capacity nnz.  Rows are compacted and sorted by
 * neighbour id; the sums are taken in a fixed order, so the result does not
 * depend on scheduling.  *nnz_out (host) receives the number of entries.
 * Stateless. */
leiden_status leiden_aggregate(int64_t n, const int64_t *offsets, const int32_t *indices,
                               const float *weights, const int32_t *membership, int64_t ncomm,
                               int64_t *out_offsets, int32_t *out_indices, float *out_weights,
                               int64_t *nnz_out, void *stream);

/* State access.  get_graph copies the current CSR (capacity n+1 / nnz; *nnz
 * host, may be queried first with NULL arrays).  get_state copies C (n
 * int32), K and Sigma (n float64 each) and 2m (host); any pointer nullable.
 * set_state installs a membership (labels in [0, n)) and recomputes K,
 * Sigma and 2m from the graph. */
leiden_status leiden_get_graph(leiden_handle *h, int64_t *offsets, int32_t *indices, float *weights,
                               int64_t *nnz /* host */, void *stream);
leiden_status leiden_get_state(leiden_handle *h, int32_t *membership, double *K, double *Sigma,
                               double *m2 /* host */, void *stream);
leiden_status leiden_set_state(leiden_handle *h, const int32_t *membership, void *stream);

int64_t leiden_num_vertices(const leiden_handle *h);
int64_t leiden_num_entries(const leiden_handle *h);

const char *leiden_strerror(int32_t status);
const char *leiden_last_error(const leiden_handle *h);

#ifdef __cplusplus
}
#endif

#endif /* LEIDEN_H */
