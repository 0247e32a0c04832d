/*
 * escape.h -- C ABI of the MI355X (gfx950) exact 4- and 5-vertex subgraph
 * counter.
 *
 * Method: Pinar, Seshadhri, Vishal, "ESCAPE: Efficiently Counting All
 * 5-Vertex Subgraphs" (arXiv 1610.09411).  The input is a simple undirected
 * graph (Sec. 2.1, problem statement); the output is, for every pattern on k
 * vertices (k = 4 or 5), the number of k-vertex subsets whose induced subgraph
 * is that pattern (Sec. 2.1; induced counts come from non-induced ones through
 * the matrix of Appendix B, disconnected patterns through Appendix A).
 *
 * Counts are exact unsigned integers.  Every step runs on the GPU: the
 * degree-ordered DAG (Sec. 2.2), the enumeration of triangles, wedges,
 * 4-cycles and 4-cliques (Thms 4vertex-tri, 4cycle, 4clique), the cut-formula
 * sums (Thms 5cutvertex, 5cutedge, 5cuttri, 5cutwed, 5formula), 5-cycles
 * (Thm 5cycle), 5-cliques (Thm 5clique) and the final linear map.
 *
 * Output order (45 slots for k = 5; the first 11 alone for k = 4):
 *   [0..5]   connected 4-vertex: 3-star, 3-path, tailed triangle, 4-cycle,
 *            diamond, 4-clique (the 4-vertex row of Fig. 5vertex)
 *   [6..10]  disconnected 4-vertex: independent set, only edge, matching,
 *            only wedge, only triangle (Fig. 4vertex-disc)
 *   [11..31] connected 5-vertex patterns 1..21 (Fig. 5vertex)
 *   [32..42] disconnected 5-vertex patterns (1)..(11) (Fig. 5vertex-disc)
 *   [43]     wedge plus a disjoint edge, [44] triangle plus a disjoint edge
 *            (the two disconnected 5-vertex graphs the figure leaves out)
 *
 * Threading: one context per host thread (calls on one context are
 * serialised by the caller).  No call throws; every error is a status code.
 */
#ifndef ESCAPE_H
#define ESCAPE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct esc_ctx esc_ctx;

/* Exact count, little-endian 128-bit: value = hi * 2^64 + lo. */
typedef struct {
    uint64_t lo, hi;
} esc_u128;

typedef enum {
    ESC_OK = 0,
    ESC_EINVAL = 1,      /* bad argument: null pointer, k not 4/5, n < 0, ... */
    ESC_ENOTSIMPLE = 2,  /* input not a simple undirected graph in sorted CSR:
                            self-loop, duplicate, unsorted row, asymmetric */
    ESC_ERANGE = 3,      /* a column id outside [0, n), or row_ptr not monotone */
    ESC_ENOMEM = 4,      /* device allocation failed or exceeds the context budget */
    ESC_EDEVICE = 5,     /* a HIP runtime call failed */
    ESC_EOVERFLOW = 6,   /* a count does not fit the requested output width */
    ESC_EBUSY = 7        /* the server's queue is full (esc_submit); retry later */
} esc_status;

/* Flags for esc_count_subgraphs. */
enum {
    ESC_F_VALIDATE = 1,        /* check the CSR on the device (ESC_ENOTSIMPLE /
                                  ESC_ERANGE on failure); without it the input
                                  must already be simple, sorted and symmetric */
    ESC_F_CANONICALIZE = 2,    /* esc_count_subgraphs only: take any CSR (rows
                                  unsorted, repeated entries, self-loops, edges
                                  listed in one row only; row_ptr[n] may be odd)
                                  and count the simple undirected graph it
                                  describes: every entry (u,v), u != v, is the
                                  edge {u,v}.  Done on the device; ids must be
                                  in [0,n) (else ESC_ERANGE).  Not accepted by
                                  esc_count_fragments or esc_count_batched
                                  (ESC_EINVAL) */
    ESC_F_INPUT_ON_DEVICE = 4, /* row_ptr / col are device pointers */
    ESC_F_RANDOM_ORDER = 8,    /* orient by a seeded pseudo-random total order
                                  instead of the degree order (test hook: counts
                                  do not depend on the order, work does) */
    ESC_F_COMPACT_LISTS = 16   /* keep the per-edge triangle lists as arc
                                  positions only (4 B per entry instead of 8;
                                  apex ids are read through the adjacency).
                                  Chosen automatically when device memory
                                  cannot hold both; same counts, slower */
};

/* Create a context on HIP device `hip_device`.  `hbm_budget_bytes` caps the
 * device memory the context may hold (0 = no cap).  On success *out owns all
 * device scratch memory; release it with esc_destroy.  Read from the
 * environment here: ESC_TRACE=1 makes the context's calls report each stage
 * (and slice) to stderr as it ends; ESC_SLICE_MS=t runs the per-source
 * kernels (4-cycles, pair passes, 5-cycles) in launches of about t ms each,
 * a workgroup taking no new task once its slice is over and the next launch
 * going on from the shared task counter (default: 30000 under ESC_TRACE,
 * else one launch; 0: one launch).  Counts do not depend on either. */
esc_status esc_create(esc_ctx **out, int hip_device, size_t hbm_budget_bytes);

/* Release every resource held by the context.  NULL is ignored. */
void esc_destroy(esc_ctx *ctx);

/* Count all induced k-vertex patterns of one graph.
 *   n        number of vertices, 0 <= n < 2^31
 *   row_ptr  n+1 int32 offsets, row_ptr[0] = 0, non-decreasing
 *   col      row_ptr[n] int32 neighbour ids: each undirected edge appears in
 *            both rows, rows sorted ascending, no self-loops, no duplicates
 *   k        4 or 5
 *   flags    ESC_F_* bits
 *   out      host array of 11 (k = 4) or 45 (k = 5) esc_u128, in the order
 *            documented above; untouched on error
 *   stream   hipStream_t to run on, or NULL for the context's own stream
 * Input arrays are read-only and not retained after return (host arrays are
 * copied to the device; device arrays are read in place).  n < k is valid: the
 * k-vertex counts are then all zero.  The call returns after the counts are on
 * the host. */
esc_status esc_count_subgraphs(esc_ctx *ctx, int32_t n, const int32_t *row_ptr,
                               const int32_t *col, int k, uint32_t flags,
                               esc_u128 *out, void *stream);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): esc_count_subgraphs with every device
 * buffer of the call taken from one fixed region of ESC_NOALLOC_SCRATCH_BYTES
 * that the library holds per GPU (a static device array, present from the
 * first use of the library on that GPU until the process ends).  The call
 * makes no hipMalloc / hipFree; the context must come from esc_create
 * (which looks the region up once per device).  Arguments, output and
 * errors as in esc_count_subgraphs; a graph whose buffers do not fit the
 * region (roughly: up to some 10^4 vertices and 10^5 edges, fewer for
 * graphs with many triangles) returns ESC_ENOMEM, with nothing retained.
 * The context's own buffers are left as they were.  All calls on one GPU
 * share the region and leave their contents in it (each call clears what
 * it needs zeroed): calls that overlap on one GPU race, so a caller
 * serialises them (one host thread, or one stream waited on between
 * calls).  Triangle lists are kept in the compact layout. */
#define ESC_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
esc_status esc_count_subgraphs_noalloc(esc_ctx *ctx, int32_t n, const int32_t *row_ptr,
                                       const int32_t *col, int k, uint32_t flags,
                                       esc_u128 *out, void *stream);

/* Same enumeration, also returning the per-vertex and per-edge fragment counts
 * of Thm 4vertex-tri, in the caller's vertex ids:
 *   tri_v, c4_v, k4_v   n uint64 each: triangles, 4-cycles and 4-cliques
 *                       containing each vertex
 *   tri_e, c4_e, k4_e   row_ptr[n] uint64 each, one per arc of the input CSR
 *                       (both arcs of an edge carry the edge's value):
 *                       triangles, 4-cycles and 4-cliques containing the edge
 * Any output pointer may be NULL.  Host memory.  Counts of the k-vertex
 * patterns go to `out` exactly as in esc_count_subgraphs. */
esc_status esc_count_fragments(esc_ctx *ctx, int32_t n, const int32_t *row_ptr,
                               const int32_t *col, int k, uint32_t flags,
                               esc_u128 *out,
                               uint64_t *tri_v, uint64_t *c4_v, uint64_t *k4_v,
                               uint64_t *tri_e, uint64_t *c4_e, uint64_t *k4_e,
                               void *stream);

/* Count all induced k-vertex patterns of each of G independent graphs in one
 * call (the method applied to every graph; Sec. 2.1 defines the counts).
 *   G        number of graphs, G >= 0 (G = 0 returns ESC_OK and does nothing)
 *   vtx_off  host, G+1 int64: graph g has vtx_off[g+1] - vtx_off[g] vertices;
 *            vtx_off[0] = 0, non-decreasing
 *   arc_off  host, G+1 int64: graph g owns col[arc_off[g] .. arc_off[g+1]),
 *            an even count (both arcs of every edge); arc_off[0] = 0
 *   row_ptr  vtx_off[G] + G int32: graph g's n_g + 1 local offsets start at
 *            row_ptr[vtx_off[g] + g], run from 0 to arc_off[g+1] - arc_off[g]
 *   col      arc_off[G] int32 local neighbour ids in [0, n_g), each graph's
 *            CSR as in esc_count_subgraphs
 *   k, flags as in esc_count_subgraphs (ESC_F_INPUT_ON_DEVICE: row_ptr and
 *            col are device pointers; vtx_off / arc_off are always host)
 *   out      host, G x (11 | 45) uint64, row g = the counts of graph g in the
 *            documented order
 *   overflow host, G bytes or NULL: overflow[g] = 1 when a count of graph g
 *            exceeds 2^64 - 1 (row g then holds the low 64 bits); with NULL,
 *            such a graph makes the call return ESC_EOVERFLOW after every row
 *            has been written
 * The sums vtx_off[G] + G and arc_off[G] must stay below 2^31.  Row offsets and
 * ids are always checked against each graph's own sizes (ESC_ERANGE); the
 * other checks follow ESC_F_VALIDATE.  Inputs are read-only and not retained;
 * the call returns after the counts are on the host.  esc_last_work then
 * reports totals over the graphs; esc_last_noninduced is not set. */
esc_status esc_count_batched(esc_ctx *ctx, int32_t G, const int64_t *vtx_off,
                             const int64_t *arc_off, const int32_t *row_ptr,
                             const int32_t *col, int k, uint32_t flags,
                             uint64_t *out, uint8_t *overflow, void *stream);

/* ------------------------------------------------------------- serving
 *
 * A request loop over the same method: jobs of any size arrive while others
 * run.  The server owns max_inflight contexts (one stream and one set of
 * device buffers each) and a worker thread per context.  A free worker takes
 * the oldest queued request and, if it has at most 2^20 vertices, the
 * following queued requests of the same k and size class up to 256 in all,
 * and runs them as one batched launch (esc_count_batched's pipeline); larger
 * requests run alone.  A group also stops growing once its predicted work
 * reaches 2^38 list visits (the wedges plus the directed 3-path bound, the
 * terms of Thm fivevertex known before counting, computed at submission), so
 * one launch does not hold many large requests.  A launch starts only when
 * its estimated device footprint (CSR and
 * arc arrays, triangle lists bounded by the wedge count, per-workgroup tables)
 * fits in the admission budget beside the launches in flight, so launches
 * overlap on the device as workers and memory free up.  Results are exact and
 * do not depend on which other requests shared a launch. */
typedef struct esc_server esc_server;

/* Start a server on ctx's device.  The admission budget is ctx's
 * hbm_budget_bytes, or half the device's free memory when that is 0.  ctx is
 * only read here; the server creates its own contexts.  max_inflight in
 * [1, 64]. */
esc_status esc_server_start(esc_ctx *ctx, int max_inflight, esc_server **out);

/* Queue a count request.  The CSR (host memory, layout as in
 * esc_count_subgraphs) is copied before return; offsets are checked here
 * (ESC_ERANGE / ESC_ENOTSIMPLE / ESC_EINVAL), the rest on the device when the
 * request runs.  *ticket identifies the request in esc_poll / esc_wait.
 * ESC_EBUSY: 2^20 requests are already waiting. */
esc_status esc_submit(esc_server *srv, int32_t n, const int32_t *row_ptr,
                      const int32_t *col, int k, uint64_t *ticket);

/* Non-blocking: *done = 0 while the request is queued or running.  Once
 * *done = 1 the request's counts (11 or 45 esc_u128, as esc_count_subgraphs)
 * are in `out`, `seconds` (nullable) holds submit-to-completion time, the
 * return value is the request's own status, and the ticket is released. */
esc_status esc_poll(esc_server *srv, uint64_t ticket, esc_u128 *out, int *done,
                    double *seconds);

/* Blocking form of esc_poll: returns when the request has completed. */
esc_status esc_wait(esc_server *srv, uint64_t ticket, esc_u128 *out, double *seconds);

/* Server counters, 8 uint64: [0] completed requests, [1] launches,
 * [2] requests that ran in batched launches, [3] peak launches in flight,
 * [4] peak estimated footprint in flight (bytes), [5] admission budget
 * (bytes), [6] requests queued now, [7] worker contexts. */
esc_status esc_server_stats(esc_server *srv, uint64_t *out);

/* Finish every queued request, stop the workers and release the server and
 * its contexts.  Tickets not yet collected are dropped. */
esc_status esc_server_stop(esc_server *srv);

/* ------------------------------------------------------------- tuning
 *
 * Launch parameters of the per-source kernels (4-cycles, pair passes,
 * wheels, 5-cycles) and of the 5-clique pass.  A context keeps a table of
 * tuned parameters keyed by the graph's degree statistics (log2 of n, of the
 * mean degree and of the largest degree, batched or not); a call uses the
 * parameters set with esc_set_params, else the table's entry for its key,
 * else the defaults.  Parameters change speed only, never counts. */
typedef struct {
    int32_t task_chunk;     /* sources taken per grab by a workgroup, 1..64
                               (default 1; 8 for batched calls) */
    int32_t wg_per_cu;      /* workgroups per CU of the per-source kernels, 1..3
                               (default 3; lowered when their tables would pass a
                               tenth of device memory) */
    int32_t k5_work_log2;   /* 5-cliques: a vertex with out-degree d is split
                               into units of min(256, 2^k5_work_log2 / d^2)
                               out-neighbours, 16..30 (default 20) */
    int32_t five_order;     /* 5-cycles of one graph (Thm 5cycle): 0 sums
                               Wnt(i,j) Y(i,j) with a table of Y (the faster
                               order) when the largest degree is below 2^16,
                               else X(i,b) Wnt(i,j) with a table of Wnt; 1
                               always the latter.  Batches always use the
                               latter.  0 or 1 (default 0) */
    int32_t k5_light;       /* 5-cliques: vertices with at most this many
                               out-neighbours (one-word rows) are counted a
                               wave each, 3..64 (default 64) */
    int32_t k5_wave_words;  /* 5-cliques: heavier vertices whose rows have at
                               most this many 64-bit words take a wave per
                               out-neighbour, the rest a workgroup per unit,
                               1..8 (default 8) */
    int32_t k5_dense_pct;   /* 5-cliques (Thm 5clique): a vertex with more than
                               k5_light and at most 4096 out-neighbours whose
                               out-neighbourhood has at least this percentage
                               of all pairs as edges is counted through the
                               complement of that neighbourhood; 0..101
                               (101: never; default 50) */
    int32_t wheel_split_deg;/* wheels (pattern 18): hubs with more neighbours
                               are split into tasks of 16 rim vertices,
                               32..2^30 (default 1024) */
    int32_t four_range_deg; /* 4-cycles (Thm 4cycle): tops with more
                               neighbours are split into key-range tasks,
                               16..2^30 (default 256) */
    int32_t pairs_hub_ranks;/* pattern 17 (Thm 5cutwed) of one graph: the
                               latest this many ranks are hubs, and the
                               diamonds with two hub tips over a dense edge
                               are summed as a matrix product of the hub /
                               dense-edge incidence; 0 (off), a multiple of
                               256 up to 65536, or -1: n / 160 rounded down
                               to a multiple of 256, at most 24576 (the
                               default).  Off for batches, for graphs with
                               fewer than twice as many vertices and when
                               its buffers would not fit the free memory */
    int32_t pairs_hub_q;    /* pattern 17: an edge is dense when at least
                               this many hubs close a triangle with it,
                               1..2^30 (default 256) */
    int32_t wheel_dense_deg;/* wheels (pattern 18) of one graph: a hub with
                               at least this many neighbours (at most 65536,
                               among the latest 65536 ranks) whose walk
                               would visit about S2/4 list entries (S2 = sum
                               of t^2 over its edges) counts its rim
                               4-cycles as (1/2) sum over rim pairs of
                               C(c,2), c = (A A)(i,j) with A the adjacency
                               of its neighbourhood, on the matrix cores
                               (4-bit float 0/1 entries, exact), when d^3/2 (d rounded up to 256) is
                               below wheel_dense_ratio * S2/4; 0 (never) or
                               4..2^30 (default 1024) */
    int32_t wheel_dense_ratio; /* multiply-adds one walk visit is worth,
                               1..2^20 (default 1024) */
    int32_t k4_dense_dplus; /* 4-cliques per triangle (Thm 4clique) of one
                               graph: a vertex a with at least this many
                               out-neighbours (and at most 65536 neighbours)
                               gets K4 of all its triangles (a,b,c), a
                               earliest, from C = B B^T on the matrix
                               cores, B the 0/1 matrix of out-neighbours b
                               by neighbours w of a, B(b,w) = [b ~ w];
                               0 (never) or 16..2^30 (default 128) */
} esc_params;

/* Time every candidate parameter set on this graph (task_chunk in {1, 4, 16}
 * x wg_per_cu in {1, 2, 3}; then, one field at a time from the best so far,
 * four_range_deg in {128, 1024}, k4_dense_dplus in {0, 1024}, and for
 * k = 5 k5_work_log2 in {22, 26},
 * k5_dense_pct in {25, 101}, k5_light in {32}, k5_wave_words in {4},
 * wheel_split_deg in {256, 4096}, pairs_hub_ranks in {0, 4096, 16384} and
 * wheel_dense_deg in {0, 4096};
 * the other fields at their defaults),
 * keep the fastest (total device time of the call) in the context's table
 * under the graph's key and return it in *best, its time in *best_ms
 * (nullable).  Arguments as in esc_count_subgraphs. */
esc_status esc_tune(esc_ctx *ctx, int32_t n, const int32_t *row_ptr, const int32_t *col, int k,
                    uint32_t flags, esc_params *best, float *best_ms, void *stream);

/* The same for a batch (arguments as in esc_count_batched, without outputs). */
esc_status esc_tune_batched(esc_ctx *ctx, int32_t G, const int64_t *vtx_off, const int64_t *arc_off,
                            const int32_t *row_ptr, const int32_t *col, int k, uint32_t flags,
                            esc_params *best, float *best_ms, void *stream);

/* Force these parameters on every later call of the context (NULL: back to
 * the table and the defaults).  ESC_EINVAL when a field is out of range. */
esc_status esc_set_params(esc_ctx *ctx, const esc_params *params);

/* Parameters the last successful call ran with. */
esc_status esc_last_params(const esc_ctx *ctx, esc_params *out);

/* Work counters of the last successful call on this context (Thm fourvertex
 * and Thm fivevertex state the running time in these terms; Fig. predict
 * fits the 5-vertex time as a linear function of W, D, DP and DBP):
 *   [0] W++  out-wedges of the DAG      [1] W+-  in-out wedges
 *   [2] W    wedges                     [3] T    triangles
 *   [4] D    diamonds                   [5] max out-degree
 *   [6] n    vertices                   [7] m    edges
 *   [8] DP   directed 3-paths i <- a -> b -> j of the DAG (four distinct
 *            vertices; the paths of the 5-cycle count, Thm 5cycle)
 *   [9] DBP  directed bipyramids: pairs of common out-neighbours of the
 *            triangles a < b < c (the 5-clique enumeration of Thm 5clique
 *            read from the triangle of the three earliest vertices); 0 for
 *            k = 4 calls, whose 5-clique pass does not run
 * Totals over the graphs of a batched call.  `out` is a host array of
 * ESC_WORK_COUNTERS uint64. */
#define ESC_WORK_COUNTERS 10
esc_status esc_last_work(const esc_ctx *ctx, uint64_t *out);

/* Non-induced counts of the last successful call (the number of subgraphs,
 * not necessarily induced, isomorphic to each pattern; Sec. 2.1), same order
 * and length as its induced output: 11 values for k = 4, 45 for k = 5.
 * `out` is a host array of that many esc_u128. */
esc_status esc_last_noninduced(const esc_ctx *ctx, esc_u128 *out);

/* Induced 3-vertex counts of the last successful esc_count_subgraphs /
 * esc_count_fragments call (the method's 3-vertex by-products, Sec. 1):
 * [0] no edge, [1] exactly one edge, [2] path (wedge), [3] triangle; they sum
 * to C(n,3).  `out` is a host array of 4 esc_u128.  Not set by batched calls. */
esc_status esc_last_three(const esc_ctx *ctx, esc_u128 *out);

/* Per-stage profile of the last successful call.  Stages, in order:
 *   [0] degree order and relabelled CSR      [1] triangles, per-arc lists
 *   [2] 4-cycles                             [3] 4-cliques per triangle and
 *                                                the triangle-cut sums
 *   [4] 5-cliques                            [5] vertex and edge sums
 *   [6] pattern 13/17 pair pass              [7] wheels (pattern 18)
 *   [8] 5-cycles                             [9] final combination
 * `ms_out` (10 floats, may be NULL): device milliseconds per stage (HIP
 * events on the call's stream).  `visits_out` (10 uint64, may be NULL):
 * elements the stage's main loop visited (neighbour or triangle-list entries
 * read, bitmap words for 5-cliques; 0 where not counted). */
esc_status esc_last_profile(const esc_ctx *ctx, float *ms_out, uint64_t *visits_out);

/* Split of the last successful call's stages into their walk and their
 * matrix-core product (the 4-cliques of dense out-neighbourhoods in
 * stage 3, Thm 4clique; the pattern-17 pairs of hubs in stage 6, Thm
 * 5cutwed; the wheels of dense hubs in stage 7), stages as in
 * esc_last_profile, each of the three arrays 10 entries, nullable:
 * `walk_ms` device milliseconds from the stage's start to the end of its
 * walk (the whole stage where it has no product), `product_ms` the rest of
 * the stage (rows and products), `product_macs` multiply-adds the products
 * issued (tiles of 256 x 256 over their padded depth). */
esc_status esc_last_products(const esc_ctx *ctx, float *walk_ms, float *product_ms, uint64_t *product_macs);

/* The signed inverse of the matrix that maps induced to non-induced counts
 * (Appendix B, figures A and A^-1), as the library builds and applies it:
 * 11 x 11 for k = 4, 34 x 34 for k = 5, rows and columns in the output order
 * above, row-major into the host array `out`.  Host-only (no device call);
 * ESC_EINVAL for other k or a NULL pointer. */
esc_status esc_inverse_matrix(int k, int32_t *out);

/* Human-readable text for a status code (static storage). */
const char *esc_strerror(esc_status s);

#ifdef __cplusplus
}
#endif

#endif /* ESCAPE_H */
