/*
 * maxflow.h -- C ABI of the MI355X maximum-flow / minimum-cut library.
 *
 * The library computes a maximum s-t flow and a minimum cut with the
 * synchronous parallel push-relabel method of Baumstark, Blelloch and Shun
 * (Sec. 3.1: rounds that fully discharge every active vertex against the
 * labels and excesses of the start of the round, settle conflicts between
 * adjacent active vertices with the win criterion, and apply new labels and
 * excess changes at the end of the round), interleaved with a parallel
 * global relabel (Sec. 2.1, Sec. 3: reverse breadth-first search from the
 * sink).  All arithmetic is exact integer arithmetic.
 *
 * Problem statement (Sec. 2, Eq. 1-2): directed graph G = (V, E) with
 * capacities c(v,w) >= 0, source s and sink t, s != t.  A flow obeys
 * f(v,w) <= c(v,w), conservation at every vertex other than s and t, and
 * antisymmetry f(v,w) = -f(w,v).  Its value is the net flow into t.  A
 * minimum cut (S, T) with s in S and t in T has capacity equal to the
 * maximum flow value.
 *
 * Graph format: CSR with paired reverse slots (the adjacency arrays of
 * Sec. 4.2 in which every edge knows its reverse edge).
 *   offsets[n+1]  int64, slots of tail v are offsets[v] .. offsets[v+1]-1,
 *                 offsets[0] = 0, non-decreasing, offsets[n] = slots
 *   head[slots]   int32, head w of slot (v, w), 0 <= w < n, w != v
 *   rev[slots]    int64, the paired reverse slot: rev[rev[a]] = a and
 *                 head[rev[a]] = v; an arc given in one direction only is
 *                 paired with a reverse slot of capacity 0
 *   cap[slots]    int32, c(v, w) >= 0, and cap[a] + cap[rev[a]] < 2^31
 * Limits: 2 <= n < 2^31, slots < 2^31 - 1.
 *
 * Outputs:
 *   value         int64, maximum flow value (net flow into t)
 *   flow[slots]   int32, flow[a] = cap[a] - residual[a]; flow[rev[a]] =
 *                 -flow[a]; a maximum flow (Eq. 1-2 hold); maximum flows
 *                 are not unique, so any valid one is correct
 *   sink_side[n]  uint8, 1 iff v reaches t in the final residual graph
 *                 (the smallest sink side T* of a minimum cut, which is
 *                 unique); 0 for every other vertex
 *   cut_capacity  int64, sum of cap[a] over slots from a vertex with
 *                 sink_side 0 to one with sink_side 1; equals value
 *
 * Errors: every call returns an mf_status and never aborts the process.
 * Ownership: the caller owns every buffer it passes; the library owns its
 * device workspace, which lives in the context and is freed by
 * mf_context_destroy.  A context serves one host thread at a time.
 */
#ifndef MI355X_MAXFLOW_H
#define MI355X_MAXFLOW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MF_OK = 0,
    MF_EINVAL = 1,     /* invalid argument or graph (see mf_last_error) */
    MF_ENOMEM = 2,     /* the request exceeds the context's HBM budget or device memory */
    MF_EDEVICE = 3,    /* a HIP call failed (see mf_last_error) */
    MF_ETIMEOUT = 4,   /* max_rounds reached; outputs hold a valid preflow */
    MF_EAGAIN = 5,     /* not finished yet (server poll) or no free slot */
    MF_ECANCELED = 6,  /* request canceled */
    MF_ENOTFOUND = 7,  /* unknown ticket or handle */
    MF_EINVARIANT = 8  /* MF_CHECK_INVARIANTS found a broken invariant (see mf_last_error) */
} mf_status;

/* A HIP stream (the type hipStream_t names), declared here so that the header
 * needs no HIP include.  NULL is the null stream. */
typedef struct ihipStream_t *mf_stream;

typedef struct {
    int32_t n;
    int64_t slots;
    const int64_t *offsets;
    const int32_t *head;
    const int64_t *rev;
    const int32_t *cap;
    int32_t s, t;
} mf_graph;

/* flags */
#define MF_PREFLOW_ONLY 0x1u   /* stop at the maximum preflow (Sec. 2.1); flow output not produced */
#define MF_PROFILE      0x2u   /* time the solver kernels with HIP events on the context's stream
                                  and count their algorithmic bytes */
#define MF_PERSISTENT   0x4u   /* run each phase as one persistent cooperative kernel with grid
                                  barriers instead of one launch per round and breadth-first level
                                  (the default); both give identical results.  On MI355X the
                                  launches are faster for one large instance: each grid barrier
                                  costs a cache write-back and invalidation per block */
#define MF_GRID_PATH    0x8u   /* solve small graphs with the grid-wide kernels too; by default a
                                  graph of at most MF_SMALL_N vertices and MF_SMALL_SLOTS slots is
                                  solved by one workgroup in a single launch (the batched form's
                                  kernel), which avoids a host round trip per round (measured
                                  faster up to about 16K slots, slower above); both give
                                  identical results */
#define MF_SIMPLE_ROUNDS 0x10u  /* rounds of the simple synchronous variant that Sec. 3 starts from
                                  (the paper's first design): every active vertex makes one pass
                                  over its arcs, pushing on every admissible arc with no win
                                  criterion, and then at most one relabel; excess changes and new
                                  labels apply at the round's end as in the default rounds.  Value,
                                  cut and sink side are the same; rounds, pushes and per-slot flow
                                  differ */
#define MF_WARM_START   0x20u  /* resume from the flow of the last complete solve of this graph on
                                  this context, after mf_graph_set_caps changed its capacities
                                  (see there): the residual state stays on the device and the
                                  solve pushes only the flow the changes allow.  Value, cut and
                                  sink side are those of the new graph.  MF_EINVAL if the context
                                  holds no resumable state for the graph.  Uses the grid-wide
                                  kernels whatever the graph's size */
#define MF_CHECK_INVARIANTS 0x40u  /* debug mode: after every round and every global relabel the
                                  solve checks the state on the device and stops with
                                  MF_EINVARIANT at the first violation: residuals >= 0 and
                                  res[a] + res[rev a] = cap[a] + cap[rev a] (the flow stays
                                  within capacity and antisymmetric, Eq. 1-2); no push left
                                  pending between rounds; every excess equals the net inflow
                                  the residuals give and is >= 0 off s (a preflow, Sec. 2.1);
                                  labels in [0, n] with d(sink) = 0 and d(excluded
                                  terminal) = n; after a global relabel also
                                  d(v) <= d(w) + 1 on every residual arc v -> w (exact
                                  distances are valid labels, Sec. 2.1).  Rounds run one per
                                  read-back in this mode, and the grid-wide kernels solve
                                  every graph */
#define MF_GAP_RELABEL  0x80u  /* the gap rule at the end of every round (Sec. 3 names gap
                                  relabeling, after Cherkassky and Goldberg, Ch. 3): when no
                                  vertex other than the terminals holds some label k in (0, n)
                                  while some hold larger ones, every label in (k, n) becomes n,
                                  for the smallest such k.  Value, cut and sink side are the same;
                                  rounds and per-slot flow differ.  Grid-wide kernels only
                                  (small graphs use them too); not in the batched and served
                                  forms, with MF_PERSISTENT or without allocation (MF_EINVAL) */
/* Batched and served forms: instances with more slots than this (by default)
 * are solved by the grid-wide kernels instead of one workgroup each. */
#define MF_BATCH_GRID_SLOTS 2097152
#define MF_SMALL_N      8192
#define MF_SMALL_SLOTS  16384

typedef struct {
    /* Global-relabel schedule (Sec. 3 and its footnote): a global relabel
     * runs when gr_freq_num * W > gr_freq_den * (gr_alpha * n + slots), where
     * W is the relabel work since the last one (each relabel of v adds
     * outdeg(v) + gr_beta) plus gr_round_charge per round.  The paper's
     * constants are freq = 1/2, alpha = 6, beta = 12 and no round charge.
     * gr_level_charge adds gr_level_charge * L to the right-hand side, L
     * being the depth of the phase's last global relabel: on a GPU a
     * relabel costs about a launch per breadth-first level, so deep
     * searches are run less often (0 = the paper's rule). */
    int64_t gr_freq_num, gr_freq_den, gr_alpha, gr_beta, gr_round_charge, gr_level_charge;
    int64_t max_rounds;          /* 0 = unlimited; counts rounds of phase 1 */
    uint32_t flags;
    int32_t lanes_per_vertex;    /* lanes that discharge one vertex: 0 = automatic, else 1..64, power of 2 */
    int32_t lanes_per_merge;     /* lanes that merge one vertex's excess: 0 = automatic */
    int32_t dense_threshold;     /* working sets above this size run in dense mode: 0 = automatic */
    int32_t blocks_per_cu;       /* persistent kernel blocks per compute unit: 0 = occupancy limit */
    int32_t lanes_per_bfs;       /* lanes that expand one frontier vertex in a top-down BFS level of
                                    the global relabel: 0 = automatic, else 1..64, power of 2 */
    uint32_t profile_mask;       /* with MF_PROFILE: kernels (bit k = mf_kernel_id k) whose launches are
                                    timed with HIP events; 0 = all.  Events cost device time, so a
                                    caller timing a solve restricts them to the kernel it studies;
                                    bytes and launch counts are kept for every kernel */
    int32_t bfs_bottom_up_factor; /* a breadth-first level of the global relabel runs bottom-up
                                    (every unlabelled vertex looks for a labelled neighbour) when
                                    frontier * factor > unlabelled vertices: 0 = automatic (8) */
    int32_t profile_stride;      /* with MF_PROFILE: time every profile_stride-th launch of each
                                    timed kernel (0 or 1 = every launch), which bounds the device
                                    time the events cost; counts and bytes cover every launch */
    int32_t check_fault_round;   /* test hook for MF_CHECK_INVARIANTS (0 = off): after this many
                                    rounds of phase 1 the host raises one residual by 1 before the
                                    check runs, which must then stop the solve with MF_EINVARIANT */
    int32_t batch_grid_slots;    /* batched and served forms: an instance with more slots than this
                                    is solved by the grid-wide kernels (one instance at a time, the
                                    whole device) instead of one workgroup (0 = MF_BATCH_GRID_SLOTS) */
    int32_t block_round_max;     /* host-driven rounds: while the working set has at most this many
                                    vertices, consecutive rounds run inside one workgroup with block
                                    barriers instead of launches per round (the same rounds, so the
                                    same results); 0 = automatic (256), negative = never.  Not used
                                    on graphs with hub vertices, with MF_CHECK_INVARIANTS or with
                                    MF_GAP_RELABEL */
    int32_t grid_workers;        /* batched form: instances above the routing size are solved by this
                                    many host threads at once, each with a stream of its own (0 = 4);
                                    the first instance's value counts for the batch */
    int32_t reserved;
} mf_options;

typedef struct {
    int64_t value, cut_capacity;
    int64_t rounds, global_relabels, bfs_levels;        /* phase 1 */
    int64_t rounds2, global_relabels2;                  /* phase 2 (flow reconstruction) */
    int64_t pushes, relabels, arc_scans, work;          /* phase 1 counters */
    double ms_preflow;   /* device time of phase 1 (init to maximum preflow) */
    double ms_total;     /* device time of the whole solve, outputs included */
    /* filled with MF_PROFILE (both phases): summed kernel durations, launch
     * counts and algorithmic bytes (the bytes the method must move: per
     * discharged vertex, slot scanned, push, merged vertex and slot, and
     * global-relabel slot and vertex) */
    double ms_discharge, ms_merge, ms_global_relabel;
    int64_t discharge_launches, merge_launches, global_relabel_launches;
    int64_t discharge_bytes, merge_bytes, global_relabel_bytes;
    /* persistent mode: summed duration and count of the phase kernel launches
     * (with MF_PROFILE the per-step times above stay 0 in this mode) */
    double ms_phase_kernel;
    int64_t phase_launches;
    /* with MF_PROFILE, per kernel (index: mf_kernel_id): summed durations of
     * its timed launches (HIP events recorded from each launch's dispatch on
     * the context's stream), number of launches and algorithmic bytes of all
     * its launches, and the number of launches timed */
    double kernel_ms[12];
    int64_t kernel_launches[12];
    int64_t kernel_bytes[12];
    int64_t kernel_timed[12];    /* launches whose durations make up kernel_ms (all of them, or
                                    every profile_stride-th one) */
    int64_t gap_lifts, gap_lifts2;   /* with MF_GAP_RELABEL: labels the gap rule set to n (phase 1,
                                        phase 2) */
} mf_stats;

/* Kernels of the host-driven path that mf_stats profiles one by one.
 * Algorithmic bytes per unit of work:
 *   discharge (list / dense): 40 per discharged vertex, 13 per slot of a
 *     discharged vertex, 16 per push;
 *   merge (list / dense): 41 per merged vertex, 4 per slot of a merged
 *     vertex, 12 per push received;
 *   flag compaction (dense rounds list their working set and their touched
 *     vertices): n per pass plus 4 per listed vertex;
 *   hub discharge / hub merge (a block per vertex of degree above 64 lanes
 *     per vertex): as discharge / merge, for the hub vertices;
 *   top-down level: 12 per frontier vertex (list entry, two offsets), 8 per
 *     slot examined (packed head with the reverse-residual bit, neighbour's
 *     label), 8 per vertex labelled;  hub expansion: 12 per hub, 12 per slot
 *     examined;
 *   bottom-up level: 4 per vertex, 8 per unlabelled vertex, 12 per slot
 *     examined, 8 per vertex labelled. */
typedef enum {
    MF_K_DISCHARGE_LIST = 0,
    MF_K_DISCHARGE_DENSE = 1,
    MF_K_MERGE_LIST = 2,
    MF_K_MERGE_DENSE = 3,
    MF_K_GR_TOPDOWN = 4,
    MF_K_GR_HUB = 5,
    MF_K_GR_BOTTOMUP = 6,
    MF_K_COMPACT = 7,
    MF_K_DISCHARGE_HUB = 8,
    MF_K_MERGE_HUB = 9,
    MF_K_BLOCK_SOLVE = 10,     /* a small graph's whole solve by one workgroup (no byte model) */
    MF_K_BLOCK_ROUNDS = 11,    /* rounds of a small working set in one workgroup (discharge and
                                  merge bytes of those rounds) */
    MF_K_COUNT = 12
} mf_kernel_id;

typedef struct mf_context mf_context;
typedef struct mf_dgraph mf_dgraph;

/* Fills *o with the paper's schedule (freq 1/2, alpha 6, beta 12, no round
 * charge), no round limit, automatic lane counts. */
void mf_options_default(mf_options *o);

/* Library version string and the last error message of a context (or of the
 * last context-free failure when ctx is NULL). */
const char *mf_version(void);
const char *mf_status_str(mf_status s);
const char *mf_last_error(const mf_context *ctx);

/* Creates a context on HIP device `device`.  hbm_budget_bytes bounds the
 * device memory the context may hold (0 = no bound beyond the device's).
 * The context owns one HIP stream on which it runs all its work. */
mf_status mf_context_create(int device, size_t hbm_budget_bytes, mf_context **out);
void mf_context_destroy(mf_context *ctx);

/* Stream ordering of the calls below that take a `stream`: the library's
 * work on the caller's device buffers is ordered after all work enqueued on
 * `stream` before the call (so a kernel that is still writing an input on
 * that stream finishes first; no device-wide synchronize is needed), and
 * work enqueued on `stream` after the call returns is ordered after the
 * library's writes to the outputs.  The calls return when their outputs are
 * complete.  `stream` must not be capturing a graph. */

/* Step 1 of a solve (residency and validation; the graph model of Sec. 2 in
 * the adjacency representation of Sec. 4.2): copies the graph into
 * library-owned device memory, narrows offsets and rev to int32 and checks
 * it (rev is an involution with matching heads, heads in range, no
 * self-loops, cap >= 0, pair sums below 2^31, s != t).  `g` holds host
 * pointers when on_device = 0 and device pointers when on_device = 1 (then
 * they must stay valid until this call returns; they are read in the order
 * of `stream`).  Returns MF_EINVAL for an invalid graph, MF_ENOMEM beyond the
 * budget. */
mf_status mf_graph_upload(mf_context *ctx, const mf_graph *g, int on_device, mf_stream stream,
                          mf_dgraph **out);
void mf_graph_free(mf_context *ctx, mf_dgraph *dg);

/* Replaces the capacities of an uploaded graph (the structure stays):
 * cap[slots] is a host array (on_device = 0) or a device array
 * (on_device = 1), checked as at upload (cap >= 0, pair sums below 2^31);
 * MF_EINVAL leaves the graph unchanged.  For re-solving a graph whose
 * capacities change between solves (vision and partitioning workloads,
 * Sec. 4 of the paper): if the context's last solve was a complete solve of
 * this graph by the grid-wide kernels (graphs small enough for the
 * one-workgroup solve need MF_GRID_PATH for it), its flow is kept on the
 * device, and a slot's residual moves by the capacity change.  *resumable (may be NULL) is then 1 if every new
 * capacity is at least the slot's flow, so that a solve with MF_WARM_START
 * can continue from that flow; otherwise 0, and the next solve starts from
 * zero flow. */
mf_status mf_graph_set_caps(mf_context *ctx, mf_dgraph *dg, const int32_t *cap, int on_device,
                            mf_stream stream, int *resumable);

/* Solves an uploaded graph: a maximum flow and a minimum cut (Sec. 2,
 * Eq. 1-2, max-flow min-cut).  Phase 1 is the synchronous push-relabel of
 * Sec. 3.1 with global relabels (Sec. 2.1, Sec. 3) up to a maximum preflow,
 * whose value is the flow value and whose residual graph gives the sink side
 * T* (Sec. 2.1); phase 2 turns the preflow into a flow by returning the
 * excess that cannot reach t to s (Sec. 2.1 second phase).  flow_dev
 * (int32[slots]) and side_dev (uint8[n]) are device pointers that receive the
 * outputs, or NULL to skip them; flow_dev must be NULL with MF_PREFLOW_ONLY.
 * The kernels run on the context's stream, ordered against `stream` as
 * stated above.  value / stats may be NULL.  MF_ETIMEOUT: max_rounds reached
 * (the outputs then describe a valid preflow); MF_EINVARIANT: see
 * MF_CHECK_INVARIANTS. */
mf_status mf_solve_uploaded(mf_context *ctx, mf_dgraph *dg, mf_stream stream, const mf_options *opt,
                            int64_t *value, int32_t *flow_dev, uint8_t *side_dev,
                            mf_stats *stats);

/* The solve of mf_solve_uploaded (same method, Sec. 2, 2.1, 3.1) for a graph
 * in host memory: upload + solve + copy-out; flow (int32[slots]) and
 * sink_side (uint8[n]) are host pointers or NULL. */
mf_status mf_solve(mf_context *ctx, const mf_graph *host_g, const mf_options *opt,
                   int64_t *value, int32_t *flow, uint8_t *sink_side, mf_stats *stats);

/* The solve of mf_solve_uploaded (same method, Sec. 2, 2.1, 3.1) for a graph
 * and outputs already in device memory (for example torch tensors), read and
 * written in the order of `stream` (see above). */
mf_status mf_solve_device(mf_context *ctx, const mf_graph *dev_g, mf_stream stream, const mf_options *opt,
                          int64_t *value, int32_t *flow_dev, uint8_t *side_dev,
                          mf_stats *stats);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): the solve of mf_solve_device with no
 * device allocation and no allocating library call.  The buffers the solve
 * needs beyond the caller's inputs and outputs (int32 copies of offsets and
 * reverse slots, and the per-solve state) live in one file-scope device
 * array of MF_NOALLOC_SCRATCH_BYTES per GPU, held from the first
 * mf_context_create on that GPU until the process ends; head and cap are
 * read in place.  A graph that needs more (about 16 bytes per slot plus 51
 * per vertex, each part rounded up to 256) gets MF_ENOMEM.  Every call on a
 * GPU shares that GPU's array, which keeps the last call's contents: calls
 * that overlap in time on one GPU (from several threads or contexts) race,
 * and the caller must not let them.  The context is created beforehand (that
 * call allocates).  Graphs of any size are solved by the grid-wide kernels;
 * MF_PROFILE and MF_WARM_START are refused (MF_EINVAL).  Arguments, stream
 * ordering, outputs and errors otherwise as mf_solve_device. */
#define MF_NOALLOC_SCRATCH_BYTES (64u << 20)
mf_status mf_solve_device_noalloc(mf_context *ctx, const mf_graph *dev_g, mf_stream stream,
                                  const mf_options *opt, int64_t *value, int32_t *flow_dev,
                                  uint8_t *side_dev, mf_stats *stats);

/* ------------------------------------------------------------------------
 * Batched solver (many instances of uneven size in one launch).
 *
 * Every instance is solved completely by one workgroup of a persistent
 * kernel that takes instances from a queue; instances are grouped by their
 * lane count (one kernel per group, on separate streams, captured together in
 * one hipGraph).  Results are identical to mf_solve's for the same options.
 */
typedef struct {
    int32_t status;              /* mf_status of this instance */
    int32_t lanes_per_vertex;    /* lane count used */
    int64_t value, cut_capacity;
    int64_t rounds, rounds2, global_relabels, global_relabels2, bfs_levels;
    int64_t pushes, relabels;
    double ms_start, ms_end;     /* batch: device time of the instance's start and end, from the
                                    first instance's start; server: device time spent pulling
                                    and checking the graph, and device time of the whole
                                    request (pull, checks, solve, results sent back) */
    double ms_latency;           /* server: time from mf_server_submit to the result being ready */
    int32_t resumed;             /* server re-solve of a resident graph: 1 if it continued from the
                                    graph's previous flow, 0 if it started from zero flow */
    int32_t reserved;
} mf_result;

/* Solves k graphs given in host memory, each by the method of
 * mf_solve_uploaded (Sec. 2, 2.1, 3.1).  Instances up to the routing size
 * (mf_options.batch_grid_slots) run in the persistent batch launch; larger
 * ones are solved while it runs by the grid-wide kernels, grid_workers of
 * them at a time (their lanes_per_vertex result is 0).  opts is NULL (the defaults for all)
 * or an array of k options (per-instance schedules, e.g. from the autotuner;
 * lanes_per_vertex 0 = automatic, otherwise 4, 8, 16 or 32).  flows[i] /
 * sides[i] are host buffers (int32[slots_i] / uint8[n_i]) or NULL, and flows
 * or sides may themselves be NULL.  An invalid graph gets MF_EINVAL in its
 * result and does not stop the others.  The whole batch must fit the HBM
 * budget (MF_ENOMEM otherwise).  stats (may be NULL) receives ms_total of the
 * batch launch. */
mf_status mf_batch_solve(mf_context *ctx, int32_t k, const mf_graph *graphs, const mf_options *opts,
                         int32_t *const *flows, uint8_t *const *sides, mf_result *results,
                         mf_stats *stats);

/* ------------------------------------------------------------------------
 * Served form: requests of mixed size arrive over time; the server admits
 * them by HBM budget in arrival order, keeps each graph and its residual state
 * in device memory until it is solved, and runs admitted requests with
 * continuous batching (a request joins the running persistent kernel as soon
 * as a workgroup is free; that workgroup pulls the graph from pinned host
 * memory and sends the results back itself).  A request with more slots than
 * the routing size (mf_options.batch_grid_slots) goes to a second lane that
 * solves such requests with the grid-wide kernels, grid_workers at a time,
 * beside the persistent kernel, in slices of the same budget.  Results are identical to
 * mf_solve's for the same options.  All server calls are thread-safe.
 */
typedef struct {
    size_t hbm_budget_bytes;   /* device memory for requests, allocated once (0 = 64 GiB) */
    int32_t max_inflight;      /* requests admitted at once (0 or above 4096 = 4096) */
    int32_t idle_ms;           /* a serve kernel leaves after this long without work (0 = 20) */
    int32_t blocks_per_cu;     /* serve kernel workgroups per compute unit (0 = occupancy limit) */
    int32_t host_staging_mib;  /* pinned host memory through which graphs and results pass, in MiB
                                  (0 = the budget, at most 1 GiB); a request needs 8(n+1) + 16 slots
                                  bytes of it, each part rounded up to 256, while it is in flight */
    int32_t grid_workers;      /* requests above the routing size run on this many grid-lane threads
                                  at once, each with a stream of its own (0 = 4); re-solves of
                                  resident graphs run on the first */
    int32_t reserved[3];
} mf_server_config;

typedef struct {
    int64_t submitted, admitted, completed, canceled, rejected;
    int64_t inflight, queued;
    size_t bytes_in_use, peak_bytes;
    int64_t kernel_launches;
} mf_server_stats;

typedef struct mf_server mf_server;

mf_status mf_server_create(mf_context *ctx, const mf_server_config *cfg, mf_server **out);
/* Joins the worker, waits for the device and frees everything; results not
 * yet polled are discarded. */
void mf_server_destroy(mf_server *srv);
/* Copies the graph (host pointers) and returns a ticket at once.  A request
 * whose graph breaks the format gets MF_EINVAL, one larger than the whole
 * HBM budget or the whole host staging arena MF_ENOMEM, both in its result. */
mf_status mf_server_submit(mf_server *srv, const mf_graph *host_g, const mf_options *opt, int want_flow,
                           uint64_t *ticket);
/* MF_EAGAIN while the request is pending; otherwise fills *out (status of the
 * request in out->status), copies flow (int32[slots]) and sink_side (uint8[n])
 * if not NULL, and forgets the ticket (MF_ENOTFOUND afterwards). */
mf_status mf_server_poll(mf_server *srv, uint64_t ticket, mf_result *out, int32_t *flow, uint8_t *sink_side);
/* As mf_server_poll but waits up to timeout_ms (negative = no limit). */
mf_status mf_server_wait(mf_server *srv, uint64_t ticket, int64_t timeout_ms, mf_result *out, int32_t *flow,
                         uint8_t *sink_side);
/* A request not yet admitted completes with MF_ECANCELED at once; an admitted
 * one completes with MF_ECANCELED when its solve ends. */
mf_status mf_server_cancel(mf_server *srv, uint64_t ticket);
mf_status mf_server_get_stats(mf_server *srv, mf_server_stats *out);

/* Resident graphs: re-solves after capacity changes (the vision and
 * partitioning inputs of Sec. 4.1 are solved again and again with new
 * capacities).  mf_server_register_graph copies the graph (host pointers)
 * into the server's device region, checks it as mf_graph_upload does, and
 * returns an id once it is resident (MF_EINVAL: invalid graph; MF_ENOMEM:
 * larger than the budget).  mf_server_submit_caps queues a solve of that
 * graph with new capacities cap[slots] (host, copied; checked as
 * mf_graph_set_caps does, an invalid one completes with MF_EINVAL): the
 * capacities replace the graph's, and the solve continues from the flow of
 * the graph's previous complete solve when every new capacity still holds
 * it (out->resumed = 1), else it starts from zero flow.  Value, cut and sink
 * side are those of the graph with the new capacities either way.
 * Requests for one graph run in submission order, by the server's grid-wide
 * lane.  mf_server_release_graph frees the graph once no queued request names
 * it (MF_ENOTFOUND: unknown id). */
mf_status mf_server_register_graph(mf_server *srv, const mf_graph *host_g, uint64_t *graph_id);
mf_status mf_server_submit_caps(mf_server *srv, uint64_t graph_id, const int32_t *cap, const mf_options *opt,
                                int want_flow, uint64_t *ticket);
mf_status mf_server_release_graph(mf_server *srv, uint64_t graph_id);

#ifdef __cplusplus
}
#endif
#endif
