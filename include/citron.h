/*
 * citron.h -- C ABI of libcitron, an exact k-clique counter for one AMD
 * Instinct MI355X (gfx950).
 *
 * Method (Lonkar & Beamer, "Accelerating Clique Counting in Sparse
 * Real-World Graphs via Communication-Reducing Optimizations"):
 *   - ordering phase (Section IV, Algorithm 3): the undirected graph is
 *     oriented into a DAG by the degree ordering: u -> v iff d(u) < d(v), or
 *     d(u) == d(v) and u < v, where d is the undirected degree; out-lists
 *     keep ascending vertex-id order;
 *   - counting phase (Section III, Algorithm 2; Section V-B, Algorithm 5 and
 *     its two heuristics): for every vertex u the subgraph induced on its
 *     out-neighbours is built from sorted-list intersections, and the
 *     (k-1)-cliques of that subgraph are counted by recursion; the last
 *     level sums degrees only; subgraphs too small to hold the rest of a
 *     clique are skipped.
 *
 * Conventions for every call:
 *   - No call aborts or throws.  Each returns a citron_status (or writes one
 *     through a status pointer); a human-readable reason for the last
 *     failure on the calling thread is available from citron_last_error().
 *   - Counts are uint64_t.  A count whose exact value is >= 2^64 is
 *     returned modulo 2^64 with status CITRON_EOVERFLOW.  The flag does not
 *     depend on the order of additions: with non-negative addends some
 *     addition carries iff the exact total is >= 2^64.
 *   - Vertex ids and CSR offsets are int32_t; a graph has fewer than 2^26
 *     vertices and its undirected CSR at most 2^31 - 1 entries (that is,
 *     fewer than 2^30 undirected edges).
 *   - The calls on one graph run their device work on the stream the graph
 *     was loaded with, and those that return results to the host
 *     synchronise it.  citron_count_batch runs on a non-blocking stream the
 *     library keeps per device, the server on non-blocking streams of its
 *     own; both return results only after their work has completed.  Work
 *     the caller queued on a graph's stream is not waited for by these two:
 *     finish it before calling them.
 *   - Different graphs may be used from different host threads at once.  A
 *     graph must not be freed while another thread uses it.  Count calls on
 *     one graph from several threads are serialised by the library.
 */
#ifndef CITRON_H
#define CITRON_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct citron_graph citron_graph;    /* opaque; owns its device memory */
typedef struct citron_server citron_server;  /* opaque; borrows its graphs */
typedef int32_t citron_status;

enum {
    CITRON_OK = 0,
    CITRON_EINVAL = 1,    /* bad argument or malformed graph */
    CITRON_ENOMEM = 2,    /* device or host allocation failed */
    CITRON_EOVERFLOW = 3, /* exact count >= 2^64; value returned mod 2^64 */
    CITRON_EDEVICE = 4,   /* a HIP runtime call failed */
    CITRON_ESTATE = 5,    /* call not valid in the graph's current state */
    CITRON_EBUSY = 6      /* server: no free slot or memory; request queued */
};

/* citron_load_csr flags */
#define CITRON_DEVICE_PTRS 1u   /* row_ptr / col_idx are device pointers */

/* Largest clique size accepted by the count calls. */
#define CITRON_KMAX 32

/* Tuning of the counting phase.  Every field only changes speed, never a
 * count.  `size` must be sizeof(citron_tuning); a field left 0 takes the
 * library default.  Ranges are checked (CITRON_EINVAL outside them). */
typedef struct {
    int32_t size;
    int32_t wg_waves;        /* waves per workgroup of the count kernel: 1..8 */
    int32_t blocks_per_cu;   /* persistent count workgroups per compute unit: 1..32 */
    int32_t light_rows;      /* rows per workgroup item of the subgraph build
                                (batches of vertices with out-degree <= 64):
                                64..1024, a multiple of 64 */
    int32_t flush_rows;      /* one-word subgraph rows a wave queues before it
                                searches them: 64..256 (at most the queue's
                                128 rows take effect) */
    int32_t build_blocks_per_cu; /* persistent build workgroups per compute
                                unit: 1..16 */
    int32_t split_pct;       /* scale of the number of parts a heavy arc or a
                                light vertex is split into, percent: 25..400
                                (schedule of a graph's counts; set it on the
                                graph, a batch uses each graph's own) */
    int32_t arc_lds_max;     /* subgraph representation switch: nodes with at
                                most this many candidates (and more than 64)
                                are copied to LDS, larger ones are walked in
                                device memory: 64..256, or 0 (the default)
                                to let the library choose by k (256 for
                                k <= 5, 224 for k = 6, 192 above: the copy's
                                LDS bounds the waves per CU) */
} citron_tuning;

/* ------------------------------------------------------------- graphs */

/* Load a simple undirected graph given as CSR and copy it to the device.
 *   n        number of vertices, 0 <= n < 2^26 (the ordering kernels run
 *            one 64-wide wave per vertex in a single dispatch)
 *   nnz      number of CSR entries = 2m (each undirected edge twice)
 *   row_ptr  int32[n+1], row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz
 *   col_idx  int32[nnz]; row u lists the neighbours of u strictly
 *            ascending; no self-loops; the graph must be symmetric
 *            (v in row u iff u in row v) -- the input of Section IV
 *   flags    0: host pointers; CITRON_DEVICE_PTRS: device pointers
 *   stream   hipStream_t used for all device work on this graph, NULL for
 *            the default stream
 *   out      receives the handle (state LOADED)
 * The arrays are only read during the call; the library keeps its own
 * copies.  Validation of every rule above runs on the device; a violation
 * gives CITRON_EINVAL and no handle. */
citron_status citron_load_csr(int32_t n, int64_t nnz, const int32_t* row_ptr,
                              const int32_t* col_idx, uint32_t flags, void* stream,
                              citron_graph** out);

/* Ordering phase (Section IV, Algorithm 3): build the degree-ordered DAG on
 * the device.  LOADED -> ORDERED; calling it again is a no-op. */
citron_status citron_order(citron_graph* g);

/* Ordering phase with the core (degeneracy) ordering instead (Section III,
 * Algorithm 1; the paper's Section IV explains why it gives the smallest
 * largest out-degree and why it is sequential as written).  Algorithm 1
 * removes one vertex of smallest current degree at a time; this call runs
 * its level-synchronous form on the device: with a threshold t starting at
 * the smallest degree, each round removes every vertex still present whose
 * current degree is <= t, then lowers its neighbours' degrees; t rises to
 * the smallest degree present when no vertex is left at or below it.
 * Vertices are ordered by (round, id) and arcs go from earlier to later,
 * so every out-degree is at most the degeneracy (the largest out-degree
 * equals it, as with Algorithm 1), while the order itself may differ from
 * Algorithm 1's one-at-a-time order.  Out-lists keep ascending id order.
 * LOADED -> ORDERED; no-op if already ordered this way, CITRON_ESTATE if
 * already ordered by degree.  Counts do not depend on the ordering; per-arc
 * counts and citron_get_dag follow it. */
citron_status citron_order_core(citron_graph* g);

/* The order key of an ORDERED graph: key (host int32[n]) receives the
 * degree of each vertex under the degree ordering, or the round in which it
 * left the peeling under the core ordering (ties broken by id in both);
 * *rounds (may be NULL) the number of peeling rounds (0 for the degree
 * ordering). */
citron_status citron_get_order_key(const citron_graph* g, int32_t* key, int32_t* rounds);

/* Counting phase: number of k-cliques of the graph, 1 <= k <= CITRON_KMAX.
 * k = 1 gives n, k = 2 gives m.  Requires ORDERED (else CITRON_ESTATE).
 * Returns 0 on error; on CITRON_EOVERFLOW returns the count mod 2^64.
 * The first count with k >= 3 builds the graph's subgraph rows (kept for
 * later counts): CITRON_EINVAL if a DAG out-degree exceeds 4096 or the rows,
 * the sum over vertices of d(u) * ceil(d(u)/64) 64-bit words with d(u) the
 * out-degree, reach 2^31 words; CITRON_ENOMEM if they do not fit in device
 * memory.  st may be NULL. */
uint64_t citron_count(citron_graph* g, int32_t k, citron_status* st);

/* The same count with the paper's own unit of work (Section III,
 * Algorithm 2 run per vertex, the subgraph of Algorithm 5 built once per
 * vertex): every vertex u with out-degree >= k - 1 is one work item whose
 * search starts at u itself and walks u's arcs in turn, with no vertex or
 * arc split across waves.  An ablation of the edge-rooted unit and the
 * heavy-arc split of citron_count, which it must equal; arguments, errors
 * and overflow as for citron_count (here k = 3 also runs the kernel). */
uint64_t citron_count_vertex_rooted(citron_graph* g, int32_t k, citron_status* st);

/* As citron_count, and also writes per_arc[e] = the number of k-cliques
 * whose two lowest vertices in the degree ordering are the endpoints of
 * DAG arc e (the order of citron_get_dag), for 2 <= k <= CITRON_KMAX.
 * per_arc is a device pointer to m uint64_t; the sum of per_arc is the
 * count.  Each entry wraps mod 2^64 on its own. */
uint64_t citron_count_per_arc(citron_graph* g, int32_t k, uint64_t* per_arc,
                              citron_status* st);

/* One of nparts disjoint shares of citron_count(g, k): the work items
 * part, part + nparts, part + 2 nparts, ... of the count's cost-ordered
 * schedule (each item is one part of a heavy arc or of a light vertex; the
 * k-cliques are the sum over arcs of Section III-B's edge-rooted counts, so
 * the shares add up to the count, mod 2^64).  The schedule breaks every
 * tie by vertex or arc id, so it depends on the graph and the tuning only:
 * shares taken by different handles of one graph, in one process or in
 * several, also add up to the count.  For progress reporting and for
 * splitting a long count over several calls.  0 <= part < nparts,
 * else CITRON_EINVAL; k <= 3 and trivial k give the whole value in part 0
 * and 0 elsewhere.  Synchronous on the graph's stream. */
uint64_t citron_count_part(citron_graph* g, int32_t k, int32_t part, int32_t nparts, citron_status* st);

/* Edge-rooted counts of selected arcs (Section III-B: the k-cliques rooted
 * at an edge are the (k-2)-cliques of the subgraph induced by the common
 * out-neighbours of its endpoints): out[i] = the number of k-cliques whose
 * two lowest vertices in the degree ordering are the endpoints of DAG arc
 * arcs[i], 2 <= k <= CITRON_KMAX.  arcs (int32[n], arc indices in
 * citron_get_dag order, each in 0..m-1, repeats allowed) and out (uint64[n])
 * are device pointers owned by the caller; 0 <= n <= 2^26.  The count kernel
 * runs in its usual launch configuration over the listed arcs only, heavy
 * ones split into parts as in a full count.  Returns the sum of out
 * (mod 2^64); *st = CITRON_EINVAL for an index outside 0..m-1 (checked on
 * the device before any count), CITRON_EOVERFLOW if the sum wrapped. */
uint64_t citron_count_arcs(citron_graph* g, int32_t k, const int32_t* arcs, int32_t n,
                           uint64_t* out, citron_status* st);

/* k-clique listing for selected arcs (the paper's conclusion: listing is a
 * small change of the counting recursion; Section III-B's edge-rooted unit):
 * for each arcs[i] = u -> v, every k-clique whose two lowest vertices in
 * the ordering are u and v, written as k vertex ids in increasing order of
 * the ordering (u, v, then one vertex per recursion level); the cliques of
 * an arc follow the depth-first order that takes each level's candidates
 * by ascending id.  2 <= k <= 16.
 *   arcs      device int32[n_arcs], arc indices in citron_get_dag order
 *             (each 0..m-1, else CITRON_EINVAL), 0 <= n_arcs <= 2^26
 *   offsets   device int64[n_arcs+1], written: the cliques of arc i are
 *             cliques[offsets[i] .. offsets[i+1]) (exclusive scan of the
 *             arcs' exact counts); written even when the output is too small
 *   cliques   device int32[cap * k], written (may be NULL with cap = 0)
 *   total     host: the number of cliques of all listed arcs
 * Returns CITRON_ENOMEM, writing no clique, when total > cap (call with
 * cap = 0 to size the buffer); CITRON_EDEVICE if the listing disagrees
 * with the count (never expected: both are exact).  Synchronous on the
 * graph's stream.  The output is 4k bytes per clique: large graphs are
 * listed by ranges of arcs. */
citron_status citron_list_arcs(citron_graph* g, int32_t k, const int32_t* arcs, int32_t n_arcs,
                               int64_t* offsets, int32_t* cliques, int64_t cap, int64_t* total);

/* Many (graph, k) queries in one persistent launch, replayed from a
 * captured HIP graph when the same query set is submitted again.  All
 * graphs must be ORDERED and share one device.  counts and sts are host
 * arrays of nq entries; sts may be NULL.  t may be NULL for the defaults.
 * Returns CITRON_OK if every query succeeded, else the first failing
 * status (the other queries still complete). */
citron_status citron_count_batch(citron_graph* const* gs, const int32_t* ks, int32_t nq,
                                 uint64_t* counts, citron_status* sts,
                                 const citron_tuning* t);

/* Progress of the citron_count_batch launch running now (for a thread
 * other than the one that called citron_count_batch): *items_taken = work
 * items claimed so far by the launch's waves (in steps of 512),
 * *items_total = its items; both 0 when no batch launch is running.  The
 * kernel stores its progress into a host-mapped word, so this call makes
 * no HIP call and never waits for the device. */
citron_status citron_batch_progress(int32_t* items_taken, int32_t* items_total);

/* Copy the DAG to host memory: dag_ptr int32[n+1], dag_col int32[m], in
 * the arc order of Algorithm 3 (rows by source id, each row ascending), for
 * whichever ordering the graph was ordered by. */
citron_status citron_get_dag(const citron_graph* g, int32_t* dag_ptr, int32_t* dag_col);

/* Sizes of a graph.  Any output pointer may be NULL.  max_outdeg is -1
 * before citron_order. */
citron_status citron_graph_info(const citron_graph* g, int64_t* n, int64_t* m,
                                int32_t* max_outdeg, int64_t* device_bytes);

/* Per-graph tuning (copied).  NULL restores the defaults.  Zero fields
 * take their defaults (wg_waves 2, blocks_per_cu 8, light_rows 256,
 * flush_rows 128, build_blocks_per_cu 4, split_pct 100, arc_lds_max chosen
 * by k).
 * A change of split_pct gives later counts a new schedule; work already
 * admitted by a server or captured in a batch keeps the schedule it was
 * built with (superseded schedules stay allocated until citron_free), so a
 * change at any time is safe and never alters a count. */
citron_status citron_set_tuning(citron_graph* g, const citron_tuning* t);
citron_status citron_get_tuning(const citron_graph* g, citron_tuning* t);

/* Work counters of one k, measured by an instrumented launch of the count
 * kernel (not a timed path).  stats receives CITRON_NSTATS uint64:
 *   [0] subgraphs built (vertices)       [1] rows built (arcs)
 *   [2] out-list entries read by the build (sum over arcs u->v of d->(v))
 *   [3] last-level AND+popcount row-word operations
 *   [4] recursion nodes pushed
 *   [5] bytes of the DAG read by the build: 4 (d->(u) + 2) per built
 *       vertex + 4 (d->(v) + 2) per built arc
 *   [6] search steps on multi-word masks (a whole wave per step)
 *   [7] nodes compacted to one word per row   [8] rows they produced
 *   [9] light-engine loop iterations (per wave)
 *   [10] sum over those iterations of the lanes holding work, so that
 *        [10] / (64 [9]) is the engine's lane occupancy
 *   [11] units started by the light engine   [12] task-buffer flushes
 *   [13] last-level candidates on multi-word masks   [14] light pops
 *   [15] sum over the kernel's waves of their busy time, [16] earliest
 *        wave start, [17] latest wave end, [18] number of waves; times in
 *        ticks of the 100 MHz device wall clock, so that
 *        1 - [15] / ([18] ([17] - [16])) is the idle-wave fraction
 *   [19] heavy arcs searched from an LDS copy of their subgraph
 *   [20] children with two levels left handled whole by one lane
 *   [21] work donations taken by idle lanes of the light engine
 *   [22] longest busy time of one wave (ticks)
 *   [23] longest single work item: (ticks << 32) | its index in the launch
 *   [24] (scratch: waves resident at the end, 0)
 *   [25] most waves resident at once
 *   [26] shader-clock cycles of all waves, start to end; of these,
 *        [27] in the light engine, [28] copying or compacting subgraphs,
 *        [29] in lane-per-child two-level searches
 *   [30] nodes finished by lane-per-child two-level searches, [31] their
 *        row-word operations had their rows been ceil(c / 64) words wide */
#define CITRON_NSTATS 32
citron_status citron_work_stats(citron_graph* g, int32_t k, uint64_t* stats);

void citron_free(citron_graph* g);       /* NULL is a no-op */

/* Reason for the last failure on this thread; valid until the next call. */
const char* citron_last_error(void);

/* Device properties used for scheduling: compute units, LDS bytes per
 * workgroup, name (up to 63 chars + NUL).  Any pointer may be NULL. */
citron_status citron_device_info(int32_t* cus, int32_t* lds_bytes, char* name64);

/* ------------------------------------------------------------ serving */

/* A request loop over resident graphs with continuous batching: requests
 * that arrive while others run are admitted as soon as a slot and device
 * memory are free, and their work overlaps on the device with the work
 * already running.  Small requests (few work items) are batched whole into
 * steps of a fast lane; each larger request runs as steps of its own, two
 * at a time on two streams.  Results do not depend on the mix a request is
 * served in.  One server drives one device from one host thread of its own. */
typedef struct {
    uint64_t tag;        /* the caller's tag from citron_server_submit */
    int32_t graph_id;
    int32_t k;
    uint64_t count;
    citron_status status;
    int32_t pad;
    int64_t t_submit_ns; /* steady-clock timestamps, nanoseconds */
    int64_t t_admit_ns;
    int64_t t_done_ns;
} citron_result;

/* hbm_budget_bytes bounds the device memory the server may hold for
 * admitted requests beyond their resident graphs: a request holds its
 * descriptor and accumulator (a few hundred bytes) and, for k > 12, its
 * share of the search stacks kept in device memory.  A request that can
 * never fit is returned with CITRON_ENOMEM; one that does not fit now waits.
 * max_slots bounds the requests in flight (1..1024). */
citron_server* citron_server_create(int64_t hbm_budget_bytes, int32_t max_slots,
                                    const citron_tuning* t);
/* Register an ORDERED graph (borrowed; must outlive the server). */
citron_status citron_server_add_graph(citron_server* s, citron_graph* g, int32_t* graph_id);
/* Queue a request; never blocks. */
citron_status citron_server_submit(citron_server* s, int32_t graph_id, int32_t k,
                                   uint64_t tag);
/* Move up to max finished results into results[]; returns how many. */
int32_t citron_server_poll(citron_server* s, citron_result* results, int32_t max);
/* Requests submitted but not yet returned by poll. */
int32_t citron_server_pending(citron_server* s);
void citron_server_destroy(citron_server* s);

/* ------------------------------------------------- no-allocation path */

/* The ordering phase for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same result as citron_load_csr + citron_order +
 * citron_get_dag, written into the caller's device buffers:
 *   n, nnz, row_ptr, col_idx  a device CSR as for citron_load_csr (device
 *            pointers, validated on the device by the same rules; EINVAL
 *            on a violation); 0 <= n <= 2^22
 *   dag_ptr  device int32[n+1], dag_col device int32[nnz/2]: the DAG in the
 *            order of citron_get_dag
 *   max_outdeg  host int32: the largest out-degree
 *   stream   hipStream_t (NULL = default); the call synchronises it
 * Working memory (out-degrees, scan partial sums, flags) is one static
 * device array of about 16.8 MB per device, held until the process ends;
 * no hipMalloc, hipFree or allocating library routine is called.  Calls
 * on one device are serialised by the library (they would otherwise race
 * on the shared array); n above 2^22 gives CITRON_EINVAL. */
citron_status citron_order_noalloc(int32_t n, int64_t nnz, const int32_t* row_ptr,
                                   const int32_t* col_idx, int32_t* dag_ptr, int32_t* dag_col,
                                   int32_t* max_outdeg, void* stream);

/* ------------------------------------------------------------ testing */

/* Test hook: the next count on g starts its accumulator at `base` instead
 * of 0 (so that the overflow flag can be forced from the host). */
citron_status citron_test_seed_accumulator(citron_graph* g, uint64_t base);

#ifdef __cplusplus
}
#endif
#endif /* CITRON_H */
