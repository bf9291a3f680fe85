/*
 * amlm.h -- C ABI of the MI355X (gfx950) temporal pattern miner.
 *
 * Given a temporal transaction multigraph (accounts are vertices, each
 * transaction is a directed edge src -> dst with an integer timestamp), the
 * library attaches to every edge exact uint32 counts of the laundering
 * patterns of the paper's multi-stage framework (Section 5): windowed
 * fan-out / fan-in, scatter-gather through at least k intermediates,
 * gather-scatter, and time-respecting cycles of length 2..L inside a window
 * delta.  The counts are the per-transaction features of Section 8 (Table 2:
 * for each transaction, how many instances of each pattern it belongs to).
 *
 * Definitions.  Edge i = (src_i -> dst_i, ts_i).  Self-loops (src == dst)
 * take part in no pattern (Section 6's differentiate operation removes an
 * account's edges to itself) and their rows are all zero.  For an anchor
 * edge e = (u -> v, t) the window is [t - delta, t] (Find_Start(t - delta)
 * and the break on timestamps past t, Section 6):
 *
 *   FAN_OUT(e)  out-edges of u with timestamp in [t - delta, t]
 *   FAN_IN(e)   in-edges of v with timestamp in [t - delta, t]
 *   S(e)        distinct s != v with an edge s -> u at a time in [t-delta, t)
 *   M_e(s)      distinct m with edges s -> m at time a and m -> v at time b,
 *               t - delta <= a < b <= t (with AMLM_SG_UNORDERED: a in
 *               [t - delta, t) and b in [t - delta, t], either order)
 *   SG_k(e)     number of s in S(e) with |M_e(s)| >= k   (Section 5,
 *               scatter-gather decomposition; Section 4: a threshold
 *               on how many intermediates take part)
 *   GS_k(e)     |S(e)| if |S(e)| >= k and u has at least k distinct
 *               destinations at times in (tau, t], tau being the earliest
 *               time of an edge into u from S(e) in the window; else 0
 *   CYC_l(e)    number of l-edge cycles that contain e (2 <= l <= L): edges
 *               c_1..c_l, dst(c_i) = src(c_{i+1}) cyclically, strictly
 *               increasing timestamps, ts(c_l) - ts(c_1) <= delta, all l
 *               vertices distinct (Section 5, cycle decomposition; Section
 *               6, classical temporal motifs as a special case)
 *
 * Stage outputs are vertex sets (Algorithm 1), so S, M and the gather-scatter
 * destinations count distinct accounts; FAN counts edges; cycles are edge
 * sets (parallel edges give distinct cycles).  Counts saturate: a count
 * whose exact value exceeds 2^32 - 1 (or the ceiling set by
 * amlm_graph_set_ceiling) is reported as that value.
 *
 * Output layout: counts[col * n_edges + i] for edge i, with one column per
 * requested pattern in the order FAN_OUT, FAN_IN, SG, GS, CYC_2 .. CYC_L,
 * DEG_OUT, DEG_IN, SG_PART, GS_PART, then the four SG size bins.
 *
 * Threading: a handle may be used by one host thread at a time.  Errors are
 * reported by the returned status; amlm_last_error() gives a thread-local
 * message for the last failing call on the calling thread.
 */
#ifndef AMLM_H
#define AMLM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AMLM_OK = 0,
    AMLM_E_INVALID = 1, /* bad argument: vertex id >= n_vertices, L outside 2..8,
                           k == 0, delta < 0, null pointer, unknown pattern bit */
    AMLM_E_RANGE = 2,   /* timestamp span >= 2^31 - 1 seconds */
    AMLM_E_NOMEM = 3,   /* device allocation failed or over the server's HBM budget */
    AMLM_E_DEVICE = 4,  /* a HIP runtime error; sticky: every later call on the
                           same handle (except destroy, info and status)
                           returns it */
    AMLM_E_ORDER = 5,   /* a stream batch is not strictly later than what came before */
    AMLM_E_BUSY = 6     /* no free server slot and the caller asked not to wait */
} amlm_status;

/* pattern bits */
#define AMLM_FAN_OUT 1u
#define AMLM_FAN_IN 2u
#define AMLM_SG 4u
#define AMLM_GS 8u
#define AMLM_CYCLES 16u
#define AMLM_ALL 31u
/* distinct counterparties inside the FAN windows (Section 8, Table 2's
 * Degree features beside the transaction counts): DEG_OUT(e) = distinct
 * destinations of u's out-edges with timestamp in [t - delta, t], DEG_IN(e)
 * = distinct sources of v's in-edges there.  Their columns come after the
 * cycle columns; AMLM_ALL does not include them. */
#define AMLM_DEG_OUT 64u
#define AMLM_DEG_IN 128u
/* modifier of AMLM_SG (adds no column): an intermediate m of sender s counts
 * when s -> m lies in [t - delta, t) and m -> v in [t - delta, t], in either
 * order; only the window bounds the two legs, as in Section 6's compiled
 * scatter-gather example (Section 4: per-step order is optional).  Without
 * it s -> m must come strictly before m -> v. */
#define AMLM_SG_UNORDERED 32u
/* modifier of AMLM_SG (adds no column; excludes AMLM_SG_UNORDERED): the
 * legs are ordered by phase, the integration phase after the placement phase
 * (Section 4): s counts when some split time tau has u's scatter leg and
 * those of at least k - 1 other intermediates in [t - delta, tau) and their
 * gather legs in [tau, t] (u's gather leg is the anchor).  k <= 8. */
#define AMLM_SG_PHASE 256u
/* modifier of AMLM_CYCLES (adds no column): a cycle's edges may occur in any
 * order (Section 4's anticipatory, out-of-order edges): l edges forming a
 * directed cycle through l distinct vertices whose timestamps span at most
 * delta, counted once from the edge of greatest (timestamp, edge id) and
 * credited to each of its edges. */
#define AMLM_CYC_ANY_ORDER 512u
/* participation columns (Section 8, Table 2: a transaction's feature is the
 * number of pattern instances it belongs to; Section 5's streaming
 * integration: a new edge increments every instance it takes part in).
 * A scatter-gather instance is a pair (anchor e, sender s) that SG_k(e)
 * counts, a gather-scatter instance a pair (e, s in S(e)) when GS_k(e) > 0.
 * An edge belongs to an instance when it is an edge of some realisation
 * of it (one edge per leg, order and window conditions met):
 *   SG_PART  the anchor; every s -> u in [t - delta, t); for each m in
 *            M_e(s) other than u, every s -> m in [t - delta, t) earlier
 *            than m's latest m -> v in [t - delta, t], and every such
 *            m -> v later than m's first s -> m (any of them with
 *            AMLM_SG_UNORDERED);
 *   GS_PART  s's edges into u in [t - delta, t), and u's out-edges at
 *            times in (tau, t] (the anchor among them), which belong to
 *            all |S(e)| instances of e.
 * One column for each of AMLM_SG and AMLM_GS that is requested, after the
 * DEG columns.  Requires AMLM_SG or AMLM_GS; excludes AMLM_SG_PHASE.  An
 * anchor credits edges older than itself: with an anchor range (the
 * server), those credits come back as deltas. */
#define AMLM_PART 1024u
/* size bins of AMLM_SG (Section 5's streaming passage counts scatter-gathers
 * of different sizes): four columns, after every other column, with the
 * number of s in S(e) whose |M_e(s)| is exactly k, k + 1, k + 2 and at
 * least k + 3 (they sum to SG_k(e)).  Requires AMLM_SG; excludes
 * AMLM_SG_PHASE. */
#define AMLM_SG_SIZES 2048u

/* schedules for the scatter-gather and cycle work (never change a count) */
#define AMLM_SCHED_STATIC 0u  /* anchors in time order, fixed-size blocks of
                                 anchors taken by atomic work stealing */
#define AMLM_SCHED_LEARNED 1u /* the cost model's predicted scatter-gather bytes
                                 cut each anchor heavier than the split size
                                 into sender-window slices (one work unit each)
                                 and group light anchors into small blocks;
                                 requires a trained or loaded cost model */
#define AMLM_SCHED_LENGTH 2u  /* as AMLM_SCHED_LEARNED, with the bytes estimated
                                 without the network: the anchor's sender-window
                                 length times a constant fitted on the same
                                 training labels (the ablation of the network);
                                 requires a model trained by this version */
#define AMLM_SCHED_GIVEN 3u   /* as AMLM_SCHED_LEARNED, with the caller's
                                 per-edge log1p(bytes) (amlm_graph_set_costs):
                                 true costs give the schedule's headroom */

typedef struct {
    uint32_t patterns;      /* OR of AMLM_FAN_OUT .. AMLM_CYCLES, optionally
                               AMLM_SG_UNORDERED with AMLM_SG */
    int64_t delta;          /* window length, same unit as the timestamps, >= 0 */
    uint32_t max_cycle_len; /* L, 2..8 (ignored without AMLM_CYCLES) */
    uint32_t k;             /* >= 1: SG / GS threshold (ignored without SG|GS) */
    uint32_t schedule;      /* AMLM_SCHED_* */
} amlm_params;

typedef struct amlm_graph amlm_graph;

/*
 * Build the device graph store (Section 6: the input is a temporal edge
 * list; the generated code walks neighbour lists sorted by time, finds each
 * window start by search and intersects sorted neighbour lists): validates
 * ids and the time span, then builds time-sorted out- and in-adjacency
 * (CSR / CSC), a neighbour-sorted copy of the in-adjacency and the
 * same-neighbour time links the kernels use.
 *
 * src, dst: n_edges vertex ids (< n_vertices).  ts: n_edges timestamps (any
 * int64; max - min must be < 2^31 - 1, else AMLM_E_RANGE).  amount:
 * optional, carried and ignored by every pattern (may be NULL).
 * inputs_on_device: 0 if the four pointers are host memory (copied), 1 if
 * they are device memory on the current device (read, not retained).
 * hip_stream: a hipStream_t (NULL = default stream); the call synchronises
 * that stream before returning.  n_edges may be 0 and must be < 2^32 - 1.
 * Errors: AMLM_E_INVALID (null pointer, id >= n_vertices), AMLM_E_RANGE,
 * AMLM_E_NOMEM, AMLM_E_DEVICE.  On success *out owns its device memory until
 * amlm_graph_destroy.
 */
amlm_status amlm_graph_create(const uint32_t *src, const uint32_t *dst, const int64_t *ts,
                              const float *amount, uint64_t n_edges, uint32_t n_vertices,
                              int inputs_on_device, void *hip_stream, amlm_graph **out);

/* Rebuild the same handle from a new edge list of any size (Section 6, as
 * for amlm_graph_create; device buffers are reused when they are large
 * enough).  Same arguments and errors as amlm_graph_create.  Queued on
 * hip_stream; synchronises it on return. */
amlm_status amlm_graph_rebuild(amlm_graph *g, const uint32_t *src, const uint32_t *dst,
                               const int64_t *ts, uint64_t n_edges, uint32_t n_vertices,
                               int inputs_on_device, void *hip_stream);

/* Free the handle and its device memory (synchronises the device).  NULL is
 * ignored. */
void amlm_graph_destroy(amlm_graph *g);

/* n_edges, number of non-self-loop edges (Section 6's differentiate removes
 * the others), n_vertices and the timestamp base (min ts).  Pointers may be
 * NULL. */
amlm_status amlm_graph_info(const amlm_graph *g, uint64_t *n_edges, uint64_t *n_valid,
                            uint32_t *n_vertices, int64_t *t_base);

/* The handle's sticky status: AMLM_OK, or AMLM_E_DEVICE once a HIP runtime
 * call failed inside a call on it (the handle then only supports destroy,
 * info and this call).  AMLM_E_INVALID for NULL. */
amlm_status amlm_graph_status(const amlm_graph *g);

/* Counts of later mining calls on g saturate at `ceiling` instead of
 * 2^32 - 1 (0 restores 2^32 - 1).  The paper fixes no width for the counts;
 * saturation keeps every result an order-independent function of the graph,
 * and a low ceiling lets a small graph reach it (tests).  AMLM_E_INVALID for
 * NULL. */
amlm_status amlm_graph_set_ceiling(amlm_graph *g, uint32_t ceiling);

/* Number of output columns for these parameters (0 on invalid parameters):
 * one per requested pattern of Section 5, cycles one per length 2..L. */
uint32_t amlm_num_columns(const amlm_params *p);

/*
 * Mine every edge of g (Sections 5 and 6: every pattern composed of stages,
 * evaluated for every transaction as the anchor of its instances; Section 8
 * uses the counts as per-transaction features).  counts_dev: caller-owned
 * device memory of amlm_num_columns(p) * n_edges uint32 on the graph's
 * device, layout [col][edge].  Asynchronous on hip_stream (NULL = default
 * stream): the host is not synchronised and the counts are valid once the
 * stream has reached this point.  Parameter errors (AMLM_E_INVALID) are
 * reported before any device work; the learned schedule without a cost
 * model is AMLM_E_INVALID.  The handle's scratch memory is allocated on the
 * first call (AMLM_E_NOMEM).
 */
amlm_status amlm_mine(amlm_graph *g, const amlm_params *p, uint32_t *counts_dev, void *hip_stream);

/* Stage timing with HIP events on the mining stream (no paper passage; for
 * benchmarks).  After amlm_set_timing(g, 1), every amlm_graph_rebuild /
 * amlm_mine on g records its stages; amlm_stage_times waits for the last
 * recorded events and returns milliseconds per stage in ms[8]: 0 graph
 * build, 1 anchor pass, 2 work-list compaction, 3 scatter-gather kernel,
 * 4 cycle kernel, 5 cost model inference, 6 work units of the learned
 * schedule, 7 the whole mining (first mining kernel to the last, the
 * overlapped cycle stream included); -1 for a stage that did not run. */
amlm_status amlm_set_timing(amlm_graph *g, int enable);
amlm_status amlm_stage_times(amlm_graph *g, float *ms);

/* Pin the launch shape of later amlm_mine calls on g (no paper passage; the
 * launch shape of the persistent kernels; 0 keeps the default of a field):
 * block = list items per scatter-gather work unit (clamped to [4, 16];
 * default 8 for the static schedule, 16 for the sliced ones);
 * sg_blocks, cyc_blocks = persistent grid sizes; split_bytes = learned
 * schedule only: an anchor whose predicted scatter-gather bytes exceed this
 * is cut into slices of about this size, each its own work unit (default
 * 32768).  Never changes a count.  AMLM_E_INVALID for a NULL g. */
amlm_status amlm_tune_set(amlm_graph *g, uint32_t block, uint32_t sg_blocks, uint32_t cyc_blocks,
                          uint32_t split_bytes);

/* Synchronise hip_stream (no paper passage): AMLM_E_DEVICE if the stream
 * reports a HIP error (sticky on g), or g's sticky status. */
amlm_status amlm_graph_sync(amlm_graph *g, void *hip_stream);

/*
 * amlm_mine for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same mining and the same counts, with the mining scratch taken from a
 * static device array of 64 MiB held by every GPU the library runs on,
 * instead of the handle's own buffers.  Calls no hipMalloc, hipFree or other
 * allocating routine, creates no stream or event, and runs on hip_stream
 * only.  The graph's device must be current.  Graphs whose scratch does not
 * fit (above about 850,000 edges) are rejected with AMLM_E_NOMEM before any
 * device work.  All calls on one GPU share the array: calls that overlap on
 * one GPU (concurrent streams, or threads) race and give wrong counts; run
 * them one after another.  Asynchronous like amlm_mine.
 */
amlm_status amlm_mine_static(amlm_graph *g, const amlm_params *p, uint32_t *counts_dev, void *hip_stream);

/*
 * Mining as amlm_mine, plus per-anchor byte counters in work_dev: device
 * uint64 [4][n_edges], rows
 *   0  B_io: the edge row read (src, dst, ts: 12 bytes) and its counts written
 *   1  B_sg/gs: the method's scatter-gather bytes of anchor i: its sender
 *      window, for each distinct sender s the smaller of s's scanned
 *      out-window (cut at the (k-1)-th qualifying intermediate other than u)
 *      and v's in-window, and the scatter scan of GS_k (Section 6's compiled
 *      scatter-gather example, its degree-ordered set intersection and
 *      Algorithm 1's early breaks), 8 bytes per element
 *   2  B_cyc: the method's cycle bytes of searches rooted at anchor i: slices
 *      of partial paths of depth 0 .. L-3 (12 bytes per element), one
 *      closing binary search per partial path of depth L-2 (8 ceil(log2
 *      in-degree(u)) bytes, Section 6's 4-cycle example) and 8 bytes per
 *      credited cycle edge
 *   3  the bytes the scatter-gather kernel itself reads for anchor i (the
 *      learned cost model's training label)
 * Rows 0-2 follow a canonical procedure that no schedule changes: they are
 * the roofline's algorithmic bytes.  Slower than amlm_mine (an extra
 * accounting pass); not for timing.
 */
amlm_status amlm_mine_work(amlm_graph *g, const amlm_params *p, uint32_t *counts_dev,
                           uint64_t *work_dev, void *hip_stream);

/* ---- stage-cell programs: patterns without a new kernel ----
 * Algorithm 1 composes a pattern from stages, each a for_all loop over the
 * windowed neighbours of a vertex found by an earlier stage, with the
 * operations of Section 6 (differentiate, difference, intersection) and
 * early termination.  A program here is a list of cells, interpreted per
 * anchor e = (u -> v, t) by one generic kernel.  Vertices are numbered
 * 0 = u, 1 = v, 2 + i = the vertex bound by cell i.  Every cell's window is
 * [lo, hi] with lo = t - delta (AMLM_T_WINDOW) or one past the time of the
 * edge bound by an earlier cell `tref` (AMLM_T_AFTER), and hi = t
 * (AMLM_T_THROUGH) or t - 1 (AMLM_T_BEFORE). */
#define AMLM_CELL_FOR_OUT 0u /* for_all: out-edges of vertex `node` in the window, binding their destination */
#define AMLM_CELL_FOR_IN 1u  /* for_all: in-edges of vertex `node` in the window, binding their source */
#define AMLM_CELL_PROBE 2u   /* the edges from vertex `node` to vertex `peer` in the window (the
                                intersection with one vertex, by binary search); last cell only */
#define AMLM_T_WINDOW 0u
#define AMLM_T_AFTER 1u
#define AMLM_T_THROUGH 0u
#define AMLM_T_BEFORE 1u
#define AMLM_AGG_SUM 0u        /* the cell's value: the sum of its bindings' inner values
                                  (1 per binding of the innermost loop) */
#define AMLM_AGG_AT_LEAST 1u   /* the number of bindings whose inner value is >= threshold */
#define AMLM_AGG_AT_LEAST_K 2u /* the same with threshold k (Section 4's minimum number taking part) */
typedef struct {
    uint8_t op;        /* AMLM_CELL_* */
    uint8_t node;      /* the vertex it expands (or probes from) */
    uint8_t peer;      /* AMLM_CELL_PROBE: the vertex the edges go to */
    uint8_t tlo;       /* AMLM_T_WINDOW or AMLM_T_AFTER */
    uint8_t tref;      /* AMLM_T_AFTER: the earlier loop cell */
    uint8_t thi;       /* AMLM_T_THROUGH or AMLM_T_BEFORE */
    uint8_t skip;      /* bit b: neighbours equal to vertex b are skipped (differentiate) */
    uint8_t distinct;  /* loops: each neighbour once (its first out-edge / last in-edge in the
                          window: a stage's output is a vertex set); probe: 0 or 1 edge */
    uint8_t agg;       /* AMLM_AGG_*: how a loop folds its bindings */
    uint8_t pad[3];
    uint32_t threshold;
} amlm_cell;

/*
 * Interpret a program of 1..6 cells for every edge of g as the anchor
 * (Algorithm 1, Section 6): out_dev[i] (device uint32[n_edges]) gets the
 * first cell's value for anchor i, saturating at the graph's ceiling;
 * self-loops get 0.  Invalid programs (a vertex or time reference used
 * before it is bound, a probe that is not the last cell, unknown codes) are
 * AMLM_E_INVALID before any device work.  One lane per anchor: a new
 * pattern costs no new kernel, at the price of the fixed kernels' tuning.
 * Asynchronous on hip_stream.
 */
amlm_status amlm_mine_program(amlm_graph *g, const amlm_cell *cells, uint32_t n_cells, int64_t delta, uint32_t k,
                              uint32_t *out_dev, void *hip_stream);

/* ---- batching: many independent graphs in one launch ---- */

/*
 * Batched store (no paper passage: the paper mines one graph; this holds
 * many independent ones, for example one partition per institution, in one
 * graph store with disjoint vertex ranges, so that one launch sequence mines
 * all of them).  src / dst hold each graph's LOCAL vertex ids (graph i:
 * 0 <= id < n_vertices[i]); graph i owns edges [edge_offsets[i],
 * edge_offsets[i + 1]) of the concatenated arrays (edge_offsets[0] = 0,
 * n_graphs + 1 entries).  The timestamps of all graphs together must span
 * < 2^31 - 1.  Pointers and errors as for amlm_graph_create; the call
 * synchronises hip_stream.  Destroy with amlm_graph_destroy.
 */
amlm_status amlm_batch_create(const uint32_t *src, const uint32_t *dst, const int64_t *ts,
                              const uint64_t *edge_offsets, const uint32_t *n_vertices, uint32_t n_graphs,
                              int inputs_on_device, void *hip_stream, amlm_graph **out);

/*
 * Mine every graph of a batched store with its own parameters ps[i] (the
 * patterns of Section 5 per graph): the same pattern set and schedule for
 * all, delta, L and k per graph.  counts_dev[i]: device memory of
 * amlm_num_columns(&ps[i]) * n_edges_i uint32, layout [col][edge] of graph i
 * (edge ids local to graph i).  The launch sequence (anchor pass, work
 * lists, scatter-gather and cycle kernels, split into the per-graph outputs)
 * is captured once into a hipGraph per launch signature and replayed on
 * hip_stream; parameters and output pointers are read from device memory at
 * replay, so they may change between calls.  Asynchronous like amlm_mine.
 */
amlm_status amlm_mine_batch(amlm_graph *batch, const amlm_params *ps, uint32_t *const *counts_dev,
                            void *hip_stream);

/* Number of sub-graphs of a batched store and how many hipGraph captures
 * amlm_mine_batch has made so far (no paper passage). */
amlm_status amlm_batch_info(const amlm_graph *g, uint32_t *n_graphs, uint32_t *captures);

/*
 * Autotune the mining launch shape of g (no paper passage: work-stealing
 * chunk size and grid sizes of the persistent kernels) by timed runs with
 * HIP events, keep the best on the handle, and cache it in the JSON file
 * cache_path (keyed by device, graph size and parameters; NULL = no cache).
 * A cached entry is used without timing.  For a batched store pass one
 * parameter set per graph and counts_dev as for amlm_mine_batch; otherwise
 * n_params = 1 and counts_dev[0].  chosen (may be NULL) receives {chunk,
 * sg_blocks, cyc_blocks}.  Counts written during tuning are the mining
 * results.
 */
amlm_status amlm_autotune(amlm_graph *g, const amlm_params *ps, uint32_t n_params, uint32_t *const *counts_dev,
                          const char *cache_path, void *hip_stream, uint32_t *chosen);

/* ---- learned cost model (scheduling only; never changes a count) ----
 * The paper has no learned component; its optimiser orders set operations
 * by an estimated cost (Section 6).  Here a network estimates each anchor's
 * scatter-gather work so the scheduler can cut heavy anchors into slices. */

/*
 * Train the 12 -> 64 -> 64 -> 1 MLP (BF16 weights, FP32 accumulation) on the
 * per-anchor work labels (row 3 of amlm_mine_work) of the given graphs, on
 * the GPU, with the library's own forward / backward / Adam kernels, and
 * keep it as the process-wide model.  If out_path is not NULL the weights
 * are also written there.  epochs, batch: training loop shape (0 = defaults:
 * 4 epochs, 4096).  Deterministic for a fixed seed.
 */
amlm_status amlm_costmodel_train(amlm_graph *const *train_graphs, const amlm_params *ps, uint32_t n,
                                 uint32_t epochs, uint32_t batch, uint64_t seed,
                                 const char *out_path, void *hip_stream);
/*
 * Held-out evaluation of the loaded model on graph g (no paper passage: the
 * gain test of the learned part).  For every anchor the scatter-gather
 * kernel works on, in time order: the model's predicted log1p(bytes), the
 * true log1p(bytes) counted by the plain miner (row 3 of amlm_mine_work) and
 * the sender-window length.  Host arrays of cap entries (any may be NULL);
 * *n gets the number of anchors (entries past cap are dropped).
 * Synchronises hip_stream.
 */
amlm_status amlm_costmodel_eval(amlm_graph *g, const amlm_params *p, uint64_t cap, float *pred, float *label,
                                uint32_t *window_len, uint64_t *n, void *hip_stream);
/* The length schedule's constant of the loaded model: predicted bytes per
 * sender-window entry (0 if the model file predates it). */
amlm_status amlm_costmodel_length_coef(float *coef);
/* Per-edge costs for AMLM_SCHED_GIVEN on g: device float[n_edges],
 * log1p(predicted bytes) by edge id, caller-owned and read during later
 * mining calls (NULL clears).  No paper passage. */
amlm_status amlm_graph_set_costs(amlm_graph *g, const float *log_cost_dev);

/* Load / save the process-wide model (weights, input mean and 1/std, the
 * length constant); no paper passage. */
amlm_status amlm_costmodel_load(const char *path);
amlm_status amlm_costmodel_save(const char *path);
/* Copy the loaded model out: weights[5057] (FP32 master values, flat layout
 * W1[64][12], b1[64], W2[64][64], b2[64], w3[64], b3), mean[12], inv_std[12].
 * Any pointer may be NULL.  No paper passage. */
amlm_status amlm_costmodel_get(float *weights, float *mean, float *inv_std);

/* Network primitives on host arrays (copied to and from the device; no paper
 * passage).  The weights are rounded to BF16 (nearest even) before use;
 * arithmetic is FP32.
 * amlm_mlp_forward: y[i] = f(x[i]) for standardised inputs x[n][12].
 * amlm_mlp_grad: gradient of mean_i (f(x[i]) - y[i])^2 with respect to the
 * 5057 parameters, accumulated over samples in a fixed order (deterministic);
 * *loss (may be NULL) receives the mean squared error. */
amlm_status amlm_mlp_forward(const float *weights, const float *x, uint32_t n, float *y);
/* The scheduler's inference path: the same network on the matrix cores
 * (16x16x32 BF16 MFMA tiles of 16 anchors), BF16 inputs and activations,
 * FP32 accumulation. */
amlm_status amlm_mlp_predict(const float *weights, const float *x, uint32_t n, float *y);
amlm_status amlm_mlp_grad(const float *weights, const float *x, const float *y, uint32_t n, float *grad,
                          float *loss);

/* ---- streaming server (continuous batching) ----
 * Section 5's streaming integration: a new transaction adds to the counts of
 * every pattern instance it completes, and the work stays local to the
 * instances it touches instead of recomputing the graph. */

typedef struct amlm_server amlm_server;

/*
 * A server mines each submitted batch incrementally against a sliding
 * window of the graph (Section 5, streaming): the new edges' own columns
 * come from instances that end at them; cycles closed by a new edge also
 * credit older edges, which are reported as sparse deltas.  Every search is
 * bounded above by its anchor's time, so a batch needs only the edges of the
 * last delta before it: the server keeps those (from `resident` and earlier
 * batches) in one window store, appends queued batches to it in groups and
 * drops edges that left the window, so its memory follows the window, not
 * the stream's length.  Batches must be strictly later in time than
 * everything before them (AMLM_E_ORDER otherwise), `resident` included.
 * hbm_budget_bytes bounds the device memory the batches being mined may
 * hold for their counts (0 = no bound; one batch is always admitted);
 * max_slots (1..16) bounds how many batches are mined concurrently, each on
 * its own HIP stream.  `resident` is read during this call only.
 */
amlm_status amlm_server_create(amlm_graph *resident, const amlm_params *p, uint64_t hbm_budget_bytes,
                               uint32_t max_slots, amlm_server **out);

/* Copy a batch of n host edges, order it after the previous batches
 * (Section 5, streaming) and queue it; it is mined once it is in the window
 * store and a slot and budget are free.  With 64 * max_slots batches
 * queued, blocks when wait != 0, else returns AMLM_E_BUSY.  *ticket
 * identifies the batch.  AMLM_E_INVALID for an endpoint >= n_vertices,
 * AMLM_E_RANGE for a batch spanning >= 2^31 - 1 - delta time units. */
amlm_status amlm_server_submit(amlm_server *s, const uint32_t *src, const uint32_t *dst,
                               const int64_t *ts, uint64_t n, int wait, uint64_t *ticket);

/*
 * Wait for a batch (Section 5, streaming).  new_counts_host: [ncols][n] for
 * the batch's own edges in submitted order (host memory, may be NULL).
 * Deltas for older edges: up to cap entries of (edge id, column,
 * increment), sorted by (edge id, column); *n_deltas gets the total number
 * (entries past cap are dropped; size cap generously).  Edge ids of stream
 * edges continue after the resident graph's: n_edges + running index in
 * submission order.  The batch's results are released by this call (a
 * second wait on the ticket is AMLM_E_INVALID); its timing record stays for
 * the 65536 most recently waited tickets.
 */
amlm_status amlm_server_wait(amlm_server *s, uint64_t ticket, uint32_t *new_counts_host,
                             uint64_t *n_deltas, uint64_t *delta_eid, uint32_t *delta_col,
                             uint32_t *delta_val, uint64_t cap);

/* Per-ticket timing (host wall clock, seconds): submit -> admitted to a
 * slot -> finished (no paper passage; for latency measurements). */
amlm_status amlm_server_ticket_times(amlm_server *s, uint64_t ticket, double *t_submit,
                                     double *t_admit, double *t_done);

/* Window store figures (no paper passage): edges in the current window
 * store, the most it has held, group commits and batches mined so far.
 * Pointers may be NULL. */
amlm_status amlm_server_stats(amlm_server *s, uint64_t *window_edges, uint64_t *max_window_edges,
                              uint64_t *commits, uint64_t *batches_done);

/* Write the server's streaming state to path (no paper passage: the state
 * of Section 5's streaming integration, kept across restarts): the window
 * store (the last delta of edges with their global edge ids), the latest
 * timestamp, the next edge id, n_vertices and the parameters.  Waits until
 * every submitted batch is in the store; batches still being mined are not
 * affected and their results stay with this server. */
amlm_status amlm_server_snapshot(amlm_server *s, const char *path);

/* A server started from a snapshot instead of a resident graph: the
 * snapshot's parameters and n_vertices, the given budget and slots.  Later
 * batches get exactly the results (rows, deltas and edge ids) they would
 * have had on the server that wrote the snapshot.  AMLM_E_INVALID for a
 * missing, truncated or corrupt file. */
amlm_status amlm_server_resume(const char *path, uint64_t hbm_budget_bytes, uint32_t max_slots, amlm_server **out);

/* Stop the server's slots and free everything it holds. */
void amlm_server_destroy(amlm_server *s);

/* Plain device-to-device copy of `bytes` (multiple of 16, 16-byte aligned
 * pointers) by the library's own streaming kernel: the achievable-bandwidth
 * probe and the calibration of the hardware byte counters (no paper
 * passage).  Asynchronous. */
amlm_status amlm_copy(void *dst, const void *src, uint64_t bytes, void *hip_stream);

/* Thread-local message describing the last error on this thread. */
const char *amlm_last_error(void);

/* ---- testing aids ---- */

/* The next build or mining call on g fails as if a HIP runtime call had
 * failed inside it: it returns AMLM_E_DEVICE, which stays sticky on g.
 * Exercises the sticky-error path without a real device fault. */
amlm_status amlm_graph_inject_device_error(amlm_graph *g);

#ifdef __cplusplus
}
#endif

#endif /* AMLM_H */
